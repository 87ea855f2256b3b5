// lap_block.hpp -- the Hungarian LAP solver of lap_wave.hpp with one LAP per
// block of kBlockLap threads (four wavefronts), for LAPs larger than a
// wavefront holds: thread t owns columns (and rows) t + kBlockLap*c, c < C, so
// m <= kBlockLap*C (1024 with C = 4).
//
// Same algorithm, same arithmetic, same tie-break as lap_wave.hpp (column
// reduction start, then shortest augmenting paths; Section 2.3 "LAP
// Solution"), so the results are bitwise those of the wavefront solvers and
// of the oracle.  What changes with the size:
//   * the matrix stays in global memory (m^2 doubles do not fit in LDS past
//     m of about 140); a Dijkstra step reads its row r, coalesced across the
//     block, from the L2;
//   * the step's minimum and chosen column are block-wide: each wavefront
//     reduces its lanes with DPP and lane permutes, then the four wavefront
//     results meet in LDS (two barriers per step);
//   * row potentials, the matching and the path links live in LDS, as the
//     per-group mirrors of the wavefront solver do.
#pragma once
#include <hip/hip_runtime.h>

#include "lap_wave.hpp"

namespace qap {

constexpr int kBlockLap = 256;                 // threads per LAP
constexpr int kBlockWaves = kBlockLap / 64;

// LDS of one block LAP: lu (m doubles, row potentials), lp (m ints: row of
// each column), lw (m ints: column proposals, then path links), row_free (m
// ints: rows still to insert), and the reduction slots.
struct BlockLapLds {
    double *lu;
    int *lp, *lw, *row_free;
    double *red_d;  // kBlockWaves doubles
    int *red_i;     // 2 * kBlockWaves ints
};

__host__ __device__ inline size_t block_lap_lds_bytes(int m)
{
    return (size_t)m * sizeof(double) + 3 * (size_t)m * sizeof(int) + kBlockWaves * sizeof(double) +
           2 * kBlockWaves * sizeof(int) + 16;
}

__device__ inline BlockLapLds block_lap_lds(char *base, int m)
{
    BlockLapLds s;
    s.lu = (double *)base;
    s.red_d = s.lu + m;
    s.lp = (int *)(s.red_d + kBlockWaves);
    s.lw = s.lp + m;
    s.row_free = s.lw + m;
    s.red_i = s.row_free + m;
    return s;
}

// Solve the m x m LAP whose row r starts at M + r*m (global memory), with all
// kBlockLap threads of the block.  Outputs per slot c (row and column
// j = t + kBlockLap*c): u[c], v[c], p[c] (row assigned to column j, -1 for
// j >= m); theta and steps on every thread.
template <int C>
__device__ void lap_solve_block(const double *__restrict__ M, int m, const BlockLapLds &L, double (&u)[C],
                                double (&v)[C], int (&p)[C], double &theta, int &steps)
{
    constexpr int kNone = 0x7fffffff;
    const int t = (int)threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    double minv[C];
    int way[C], prop[C];
    unsigned used = 0u, intree = 0u;
    // column reduction: every thread scans its own columns down the rows
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = t + kBlockLap * c;
        u[c] = 0.0;
        v[c] = 0.0;
        p[c] = -1;
        minv[c] = kInf;
        way[c] = -1;
        prop[c] = 0;
        if (j < m) {
            double best = M[j];
            int arg = 0;
            for (int i = 1; i < m; ++i) {
                const double x = M[(size_t)i * m + j];
                if (x < best) {
                    best = x;
                    arg = i;
                }
            }
            v[c] = best;
            prop[c] = arg;
            L.lw[j] = kNone;
            L.lu[j] = best;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (t + kBlockLap * c < m) atomicMin(&L.lw[prop[c]], t + kBlockLap * c);
    __syncthreads();
    // the LAP value starts at the left fold of the column minima
    double th = L.lu[0];
    for (int j = 1; j < m; ++j) th = th + L.lu[j];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = t + kBlockLap * c;
        if (j < m) {
            p[c] = (L.lw[prop[c]] == j) ? prop[c] : -1;
            L.row_free[j] = (L.lw[j] == kNone) ? 1 : 0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = t + kBlockLap * c;
        if (j < m) {
            L.lp[j] = p[c];
            L.lu[j] = 0.0;
        }
    }
    __syncthreads();
    int st = 0;
    int i0 = 0;
    while (i0 < m && !L.row_free[i0]) ++i0;
    while (i0 < m) {
        // one shortest augmenting path from row i0
#pragma unroll
        for (int c = 0; c < C; ++c) {
            minv[c] = kInf;
            way[c] = -1;
        }
        used = 0u;
        intree = ((i0 % kBlockLap) == t) ? (1u << (i0 / kBlockLap)) : 0u;
        int r = i0, last = -1, js;
        for (;;) {
            ++st;
            const double ur = L.lu[r];
            const double *row = M + (size_t)r * m;
            double best = kInf;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int j = t + kBlockLap * c;
                if (j < m && !((used >> c) & 1u)) {
                    const double s = (row[j] - ur) - v[c];
                    if (s < minv[c]) {
                        minv[c] = s;
                        way[c] = last;
                    }
                    best = dmin(best, minv[c]);
                }
            }
            // block minimum: wavefronts, then their four results in LDS
            best = group_min<64>(best);
            if (lane == 0) L.red_d[wave] = best;
            __syncthreads();
            double mn = L.red_d[0];
#pragma unroll
            for (int w = 1; w < kBlockWaves; ++w) mn = dmin(mn, L.red_d[w]);
            // chosen column: tied non-tree columns, unmatched first, lowest index
            int jf = kNone, ja = kNone;
#pragma unroll
            for (int c = C - 1; c >= 0; --c) {
                const int j = t + kBlockLap * c;
                if (j < m && !((used >> c) & 1u) && minv[c] == mn) {
                    ja = j;
                    if (p[c] < 0) jf = j;
                }
            }
            jf = group_min_i32<64>(jf);
            ja = group_min_i32<64>(ja);
            if (lane == 0) {
                L.red_i[wave] = jf;
                L.red_i[kBlockWaves + wave] = ja;
            }
            __syncthreads();
            int bf = L.red_i[0], ba = L.red_i[kBlockWaves];
#pragma unroll
            for (int w = 1; w < kBlockWaves; ++w) {
                bf = min(bf, L.red_i[w]);
                ba = min(ba, L.red_i[kBlockWaves + w]);
            }
            js = (bf != kNone) ? bf : ba;
            const double delta = mn;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int j = t + kBlockLap * c;
                if ((intree >> c) & 1u) u[c] = u[c] + delta;
                if (j < m) {
                    if ((used >> c) & 1u)
                        v[c] = v[c] - delta;
                    else
                        minv[c] = minv[c] - delta;
                }
            }
            th = th + delta;
            const int pj = L.lp[js];
            if (pj < 0) break;
            if ((js % kBlockLap) == t) used |= 1u << (js / kBlockLap);
            if ((pj % kBlockLap) == t) intree |= 1u << (pj / kBlockLap);
            r = pj;
            last = js;
        }
        // flip the alternating path js <- way[js] <- ... <- root: every column
        // on it takes the old row of its predecessor (the root row i0 for the
        // first column); tree rows publish their potentials
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = t + kBlockLap * c;
            if (j < m) L.lw[j] = way[c];
            if ((intree >> c) & 1u) L.lu[j] = u[c];
        }
        __syncthreads();
        unsigned onpath = 0u;
        for (int j = js; j >= 0; j = L.lw[j])
            if ((j % kBlockLap) == t) onpath |= 1u << (j / kBlockLap);
        int np[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int w = way[c];
            np[c] = (w < 0) ? i0 : L.lp[w < 0 ? 0 : w];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if ((onpath >> c) & 1u) {
                p[c] = np[c];
                L.lp[t + kBlockLap * c] = np[c];
            }
        }
        __syncthreads();
        ++i0;
        while (i0 < m && !L.row_free[i0]) ++i0;
    }
    theta = th;
    steps = st;
}

// One LAP per block (validation and large-LAP entry point, qap_lap_batch):
// LAP b's matrix at cost + b*m*m; outputs as k_lap_batch's.
template <int C>
__global__ __launch_bounds__(kBlockLap) void k_lap_block(const double *__restrict__ cost, int count, int m,
                                                         double *__restrict__ uo, double *__restrict__ vo,
                                                         double *__restrict__ tho, int *__restrict__ rco)
{
    extern __shared__ double lds_block[];
    const long long b = blockIdx.x;
    if (b >= count) return;
    const BlockLapLds L = block_lap_lds((char *)lds_block, m);
    double u[C], v[C], th;
    int p[C], st;
    lap_solve_block<C>(cost + b * (long long)m * m, m, L, u, v, p, th, st);
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = t + kBlockLap * c;
        if (j < m) {
            uo[b * m + j] = u[c];
            vo[b * m + j] = v[c];
            rco[b * m + j] = p[c];
        }
    }
    if (t == 0) tho[b] = th;
}

}  // namespace qap
