// lap_scalar.hpp -- the Hungarian LAP solver of lap_wave.hpp with its control
// held in scalar registers: a wavefront solves H independent LAPs at once
// (H = 1: one LAP on 64 lanes, m <= 64; H = 2: two LAPs on 32 lanes each,
// m <= 32).  Lane l of part h owns row l and column l of LAP h.
//
// Same algorithm, same arithmetic, same tie-break as lap_wave.hpp (column
// reduction start, then shortest augmenting paths, Section 2.3 "LAP
// Solution"; see there for the fixed choice of optimal duals), so results are
// bitwise identical.  What differs is
// the mapping: the current row, the chosen column, the matched row, the path
// and the tree/used sets of each part are wave-uniform values (SGPRs, lane
// masks), so the scalar unit runs the control flow and a Dijkstra step costs
// about forty vector instructions for all H LAPs of the wave.
#pragma once
#include <hip/hip_runtime.h>

#include "lap_wave.hpp"

namespace qap {

__device__ __forceinline__ double vmin_f64(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <int CTRL>
__device__ __forceinline__ double mov_dpp_d(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// min over each 32-lane half (RW = 32) or the whole wave (RW = 64); every
// lane receives the minimum of its half / of the wave.  Inputs are never NaN.
template <int RW>
__device__ __forceinline__ double part_min(double x)
{
    x = vmin_f64(x, mov_dpp_d<0x128>(x));  // row_ror:8
    x = vmin_f64(x, mov_dpp_d<0x124>(x));  // row_ror:4
    x = vmin_f64(x, mov_dpp_d<0x122>(x));  // row_ror:2
    x = vmin_f64(x, mov_dpp_d<0x121>(x));  // row_ror:1
    {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(x), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(x), false, false);
        x = vmin_f64(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
    }
    if constexpr (RW == 64) {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
        x = vmin_f64(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
    }
    return x;
}

__device__ __forceinline__ int sgpr(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Solve H LAPs.  All data lives in the block's LDS array `lds`: part h's
// matrix (row stride m) at lds + tile_off[h], its scratch at lds +
// scr_off[h] (m doubles: row potentials, then m ints: matching, then m ints:
// path links).  Offsets rather than pointers keep every access a known LDS
// access (a per-lane choice between generic pointers compiles to flat
// loads).  nparts <= H parts are live (the others are skipped).  Outputs for
// lane l of part h: u (row l), v (column l), p (row matched to column l, -1
// past m); theta and steps of the lane's part.  On return the scratch holds
// that part's row potentials.
// RW: width of the step's min reduction, 32 when every live column sits in
// the lower half-wave (H = 2, or H = 1 with m <= 32: the upper lanes never
// take part, and what they receive is never used), else 64.
template <int H, int RW = (H == 1 ? 64 : 32)>
__device__ void lap_solve_scalar(double *lds, const int *tile_off, const int *scr_off, int m, int nparts,
                                 double &u, double &v, int &p, double &theta, int &steps)
{
    constexpr int W = 64 / H;  // lanes per part
    const int lane = (int)(threadIdx.x & 63);
    const int h = (H == 1) ? 0 : (lane >> 5);
    const int l = lane & (W - 1);
    const bool valid = l < m && h < nparts;
    const int toff = (H == 1 || h == 0) ? tile_off[0] : tile_off[H - 1];
    const int soff = (H == 1 || h == 0) ? scr_off[0] : scr_off[H - 1];
    const double *M = lds + toff;
    double *mlu = lds + soff;
    int *mlp = (int *)(mlu + m);
    int *mlw = mlp + m;

    // column reduction: lane l scans column l of its part
    constexpr int kNone = 0x7fffffff;
    u = 0.0;
    v = 0.0;
    p = -1;
    int prop = 0;
    if (valid) {
        double best = M[l];
        for (int i = 1; i < m; ++i) {
            const double x = M[i * m + l];
            if (x < best) {
                best = x;
                prop = i;
            }
        }
        v = best;
        mlw[l] = kNone;
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) atomicMin(&mlw[prop], l);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        p = (mlw[prop] == l) ? prop : -1;
        mlp[l] = p;
        mlu[l] = 0.0;
    }
    const unsigned long long unm_all = __builtin_amdgcn_ballot_w64(valid && mlw[l] == kNone);
    __builtin_amdgcn_wave_barrier();
    double minv = kInf;
    int way = -1;
    bool used = false;
    bool intree = false;
    double th = 0.0;
    int st = 0;
    // per-part scalar state: rows still to insert, current row, last column;
    // the LAP value starts at the left fold of the part's column minima
    unsigned long long unm[H];
    int i0[H], r[H], last[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        unm[q] = (H == 1) ? unm_all : ((unm_all >> (32 * q)) & 0xffffffffull);
        i0[q] = (q < nparts && unm[q]) ? (int)__builtin_ctzll(unm[q]) : m;
        r[q] = i0[q];
        last[q] = -1;
        if (q < nparts) {
            double f = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), q * W),
                                        __builtin_amdgcn_readlane(__double2loint(v), q * W));
            for (int j = 1; j < m; ++j)
                f = f + __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), q * W + j),
                                         __builtin_amdgcn_readlane(__double2loint(v), q * W + j));
            if (H == 1 || h == q) th = f;
        }
    }
    intree = valid && i0[(H == 1) ? 0 : h] == l;
    for (;;) {
        bool any = false;
#pragma unroll
        for (int q = 0; q < H; ++q) any = any || (i0[q] < m);
        if (!any) break;
        const int my_i0 = (H == 1 || h == 0) ? i0[0] : i0[H - 1];
        const bool part_live = my_i0 < m;
        const int my_r = (H == 1 || h == 0) ? r[0] : r[H - 1];
        const int my_last = (H == 1 || h == 0) ? last[0] : last[H - 1];
        if (part_live) ++st;
        const bool act = valid && part_live && !used;
        const double ur = mlu[my_r];
        const double mv = M[my_r * m + (l < m ? l : 0)];
        const double s = (mv - ur) - v;
        if (act && s < minv) {
            minv = s;
            way = my_last;
        }
        const double mn = part_min<RW>(act ? minv : kInf);
        const bool cand = act && minv == mn;
        const unsigned long long bc = __builtin_amdgcn_ballot_w64(cand);
        const unsigned long long bf = __builtin_amdgcn_ballot_w64(cand && p < 0);
        int js[H];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const unsigned long long cq = (H == 1) ? bc : ((bc >> (32 * q)) & 0xffffffffull);
            const unsigned long long fq = (H == 1) ? bf : ((bf >> (32 * q)) & 0xffffffffull);
            js[q] = (int)__builtin_ctzll(fq != 0ull ? fq : (cq | (1ull << 63)));
        }
        if (part_live) {
            if (intree) u = u + mn;
            if (valid) {
                if (used)
                    v = v - mn;
                else
                    minv = minv - mn;
            }
            th = th + mn;
        }
        const int my_js = (H == 1 || h == 0) ? js[0] : js[H - 1];
        const int pjv = mlp[my_js < m ? my_js : 0];
        int pj[H];
#pragma unroll
        for (int q = 0; q < H; ++q) pj[q] = __builtin_amdgcn_readlane(pjv, q * W);
#pragma unroll
        for (int q = 0; q < H; ++q) {
            if (i0[q] >= m) continue;
            const bool mine = (H == 1) || (h == q);
            if (pj[q] >= 0) {
                if (mine && l == js[q]) used = true;
                if (mine && valid && l == pj[q]) intree = true;
                r[q] = pj[q];
                last[q] = js[q];
                continue;
            }
            // flip the alternating path of part q back to its root row; the
            // path links are the lanes' own `way` registers
            if (mine && valid && intree) mlu[l] = u;
            __builtin_amdgcn_wave_barrier();
            unsigned long long onpath = 0ull;
            int j = js[q];
            while (j >= 0) {
                onpath |= 1ull << j;
                j = __builtin_amdgcn_readlane(way, q * W + j);
            }
            int np = -1;
            const bool flip = mine && valid && ((onpath >> l) & 1ull);
            if (flip) np = (way < 0) ? i0[q] : mlp[way];
            __builtin_amdgcn_wave_barrier();
            if (flip) {
                p = np;
                mlp[l] = np;
            }
            __builtin_amdgcn_wave_barrier();
            unm[q] &= unm[q] - 1ull;
            i0[q] = unm[q] ? (int)__builtin_ctzll(unm[q]) : m;
            r[q] = i0[q];
            last[q] = -1;
            if (mine) {
                minv = kInf;
                way = -1;
                used = false;
                intree = valid && l == i0[q];
            }
        }
    }
    theta = th;
    steps = st;
}

// One LAP per wavefront (the H = 1 case above) with the per-column flags
// held as wave masks in SGPRs rather than per-lane booleans: the tree rows,
// the tree (used) columns and the unmatched columns.  A mask turns back into
// a lane predicate for free (inverse ballot: the SGPR pair is the lane mask
// of a v_cndmask or of exec), so the tie-break ballot is a single compare
// and the flag updates are scalar bit operations.  Non-tree work columns
// keep minv, every other lane holds +inf, so the step's minimum reads minv
// directly.  Arithmetic, order and tie-break are those of lap_solve_scalar,
// so the results are bitwise identical to it.
// Arguments as lap_solve_scalar with one part: tile at lds + toff, scratch
// at lds + soff (m doubles, then 2m ints); m <= RW.
template <int RW>
__device__ void lap_solve_scalar1(double *lds, int toff, int soff, int m, double &u, double &v, int &p,
                                  double &theta, int &steps)
{
    const int l = (int)(threadIdx.x & 63);
    const bool valid = l < m;
    const double *M = lds + toff;
    double *mlu = lds + soff;
    int *mlp = (int *)(mlu + m);
    int *mlw = mlp + m;
    const unsigned long long validm = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);

    // column reduction: lane l scans column l
    constexpr int kNone = 0x7fffffff;
    u = 0.0;
    v = 0.0;
    p = -1;
    int prop = 0;
    if (valid) {
        double best = M[l];
        for (int i = 1; i < m; ++i) {
            const double x = M[i * m + l];
            if (x < best) {
                best = x;
                prop = i;
            }
        }
        v = best;
        mlw[l] = kNone;
        mlu[l] = best;  // staged for the fold below
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) atomicMin(&mlw[prop], l);
    __builtin_amdgcn_wave_barrier();
    // the LAP value starts at the left fold of the column minima
    double th = mlu[0];
    for (int j = 1; j < m; ++j) th = th + mlu[j];
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        p = (mlw[prop] == l) ? prop : -1;
        mlp[l] = p;
        mlu[l] = 0.0;
    }
    unsigned long long unm = __builtin_amdgcn_ballot_w64(valid && mlw[l] == kNone);  // rows to insert
    unsigned long long freem = __builtin_amdgcn_ballot_w64(valid && p < 0);         // unmatched columns
    __builtin_amdgcn_wave_barrier();
    int st = 0;
    if (unm) {
        int i0 = (int)__builtin_ctzll(unm);
        int r = i0, last = -1;
        unsigned long long usedm = 0ull, treem = 1ull << i0;
        double minv = kInf;
        int way = -1;
        for (;;) {
            ++st;
            const unsigned long long actm = validm & ~usedm;
            const double ur = mlu[r];
            const double mv = M[r * m + (valid ? l : 0)];
            const double s = (mv - ur) - v;
            const unsigned long long bm = __builtin_amdgcn_ballot_w64(s < minv) & actm;
            minv = __builtin_amdgcn_inverse_ballot_w64(bm) ? s : minv;
            way = __builtin_amdgcn_inverse_ballot_w64(bm) ? last : way;
            const double mn = part_min<RW>(minv);
            const unsigned long long eqm = __builtin_amdgcn_ballot_w64(minv == mn);
            const unsigned long long bf = eqm & freem;
            const int js = (int)__builtin_ctzll(bf != 0ull ? bf : (eqm | (1ull << 63)));
            // masked adds kept as branches over exec (one VALU op each)
            // rather than if-converted to add + two selects
            if (__builtin_amdgcn_inverse_ballot_w64(treem)) asm volatile("v_add_f64 %0, %0, %1" : "+v"(u) : "v"(mn));
            if (__builtin_amdgcn_inverse_ballot_w64(usedm)) asm volatile("v_add_f64 %0, %0, -%1" : "+v"(v) : "v"(mn));
            minv = __builtin_amdgcn_inverse_ballot_w64(1ull << js) ? kInf : minv - mn;
            th = th + mn;
            const int pj = __builtin_amdgcn_readlane(p, js);
            if (pj >= 0) {
                usedm |= 1ull << js;
                treem |= 1ull << pj;
                r = pj;
                last = js;
                continue;
            }
            // flip the alternating path back to the root row; the path
            // links are the lanes' own `way` registers
            if (__builtin_amdgcn_inverse_ballot_w64(treem)) mlu[l] = u;
            __builtin_amdgcn_wave_barrier();
            unsigned long long onpath = 0ull;
            int j = js;
            while (j >= 0) {
                onpath |= 1ull << j;
                j = __builtin_amdgcn_readlane(way, j);
            }
            const bool flip = __builtin_amdgcn_inverse_ballot_w64(onpath);
            int np = -1;
            if (flip) np = (way < 0) ? i0 : mlp[way];
            __builtin_amdgcn_wave_barrier();
            if (flip) {
                p = np;
                mlp[l] = np;
            }
            __builtin_amdgcn_wave_barrier();
            freem &= ~(1ull << js);
            unm &= unm - 1ull;
            if (!unm) break;
            i0 = (int)__builtin_ctzll(unm);
            r = i0;
            last = -1;
            usedm = 0ull;
            treem = 1ull << i0;
            minv = kInf;
            way = -1;
        }
    }
    theta = th;
    steps = st;
}

}  // namespace qap
