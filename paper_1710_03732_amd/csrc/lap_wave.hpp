// lap_wave.hpp -- Hungarian LAP solver for one group of L lanes of a 64-wide
// CDNA wavefront (L in {8, 16, 32, 64}); lane l owns columns (and rows)
// l + L*c for c < C, so m <= L*C.
//
// The method: shortest augmenting paths with row/column potentials, the
// primal-dual Hungarian algorithm that solves every Z-, Y- and X-LAP of the
// three-stage decomposition of DLRLT2 (Section 2.3, "LAP Solution").  The
// paper does not say which optimal duals a solver must return; this solver
// makes the fixed choice the whole library is built on:
//   * start by column reduction: v[j] = min_i M[i][j], u = 0; every column
//     proposes the lowest row attaining its minimum and each proposed row is
//     matched to the lowest proposing column; the LAP value starts at the
//     left fold of v[0..m-1]; the unmatched rows are then inserted in
//     ascending order;
//   * a Dijkstra step scans the newest tree row r: every non-tree column j
//     computes s = (M[r][j] - u[r]) - v[j] and keeps it in minv[j] when
//     strictly smaller, remembering the column through which it was reached;
//   * the next column is the non-tree column of least minv; ties prefer an
//     unmatched column, then the lowest index;
//   * delta = that least minv; tree rows u += delta, tree columns v -= delta,
//     non-tree columns minv -= delta; the LAP value gets += delta;
//   * reaching an unmatched column flips the alternating path to the root.
// Every per-column operation is one IEEE add, subtract or compare and the
// argmin is an exact min, so the result does not depend on L or C.
//
// Cross-lane work per Dijkstra step, all without LDS round trips:
//   * min over the group: DPP row rotations inside 16-lane rows (half-row
//     mirror and quad permutes for 8-lane groups), v_permlane16_swap across
//     the two rows of a 32-lane group, v_permlane32_swap across wave halves;
//   * the chosen column: each lane offers its lowest tied column (and its
//     lowest unmatched tied one), and an integer minimum over the group by
//     the same lane moves picks the lowest index, unmatched columns first;
//   * the potential of the next row and the row matched to the chosen column
//     are read from a per-group LDS mirror (u is written back there when a
//     row's search ends, the matching when a path flips), at a group-uniform
//     address.
#pragma once
#include <hip/hip_runtime.h>

namespace qap {

constexpr double kInf = __builtin_huge_val();

// Lane moves for the group minima.  Every control used here (row
// rotations, half-row mirror, quad permutes) gives each lane a source lane,
// so the result does not depend on the old value: bound_ctrl with full masks
// needs no copy of it.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// The minimum of two doubles that are never NaN, as one v_min_f64 (fmin
// would first quiet each operand, which changes nothing here).
__device__ __forceinline__ double dmin(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// min over each 16-lane DPP row (every lane gets the row minimum)
__device__ __forceinline__ double row16_min(double x)
{
    x = dmin(x, dpp_d<0x128>(x));  // row_ror:8
    x = dmin(x, dpp_d<0x124>(x));  // row_ror:4
    x = dmin(x, dpp_d<0x122>(x));  // row_ror:2
    x = dmin(x, dpp_d<0x121>(x));  // row_ror:1
    return x;
}

// min over each 8-lane half row
__device__ __forceinline__ double half8_min(double x)
{
    x = dmin(x, dpp_d<0x141>(x));  // row_half_mirror
    x = dmin(x, dpp_d<0x4E>(x));   // quad_perm [2,3,0,1]
    x = dmin(x, dpp_d<0xB1>(x));   // quad_perm [1,0,3,2]
    return x;
}

__device__ __forceinline__ double swap16_min(double x)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(x), false, false);
    return dmin(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
}

__device__ __forceinline__ double swap32_min(double x)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
    return dmin(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
}

template <int L>
__device__ __forceinline__ double group_min(double x)
{
    if constexpr (L == 8) {
        return half8_min(x);
    } else {
        x = row16_min(x);
        if constexpr (L >= 32) x = swap16_min(x);
        if constexpr (L == 64) x = swap32_min(x);
        return x;
    }
}

// The same minimum for ints (the chosen column's index).
template <int L>
__device__ __forceinline__ int group_min_i32(int k)
{
    if constexpr (L == 8) {
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x141, 0xf, 0xf, true));  // row_half_mirror
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x4E, 0xf, 0xf, true));   // quad_perm [2,3,0,1]
        return min(k, __builtin_amdgcn_mov_dpp(k, 0xB1, 0xf, 0xf, true));  // quad_perm [1,0,3,2]
    } else {
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x128, 0xf, 0xf, true));  // row_ror:8
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x124, 0xf, 0xf, true));  // row_ror:4
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x122, 0xf, 0xf, true));  // row_ror:2
        k = min(k, __builtin_amdgcn_mov_dpp(k, 0x121, 0xf, 0xf, true));  // row_ror:1
        if constexpr (L >= 32) {
            const auto a = __builtin_amdgcn_permlane16_swap(k, k, false, false);
            k = min((int)a[0], (int)a[1]);
        }
        if constexpr (L == 64) {
            const auto b = __builtin_amdgcn_permlane32_swap(k, k, false, false);
            k = min((int)b[0], (int)b[1]);
        }
        return k;
    }
}

// Per-group LDS scratch of lap_solve: lu (m doubles), lp and lw (m ints each).
// Solve the m x m LAP whose row r starts at M + r*m (LDS).  gbase = lane of
// the group's first lane within the wavefront.  Outputs per slot c (column /
// row j = l + L*c): u[c] row potential, v[c] column potential, p[c] row
// assigned to column j (-1 for j >= m); theta = LAP value; steps = Dijkstra
// steps.  On return lu holds u.  All lanes of the group must be active.
template <int L, int C>
__device__ void lap_solve(const double *__restrict__ M, int m, int l, int gbase, double *lu, int *lp,
                          int *lw, double (&u)[C], double (&v)[C], int (&p)[C], double &theta,
                          int &steps)
{
    static_assert(L == 8 || L == 16 || L == 32 || L == 64, "group size");
    const unsigned long long gmask = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << gbase);
    constexpr int kNone = 0x7fffffff;
    double minv[C];
    int way[C], prop[C];
    unsigned used = 0u, intree = 0u;
    // column reduction: each lane scans its own columns (conflict-free LDS reads)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = l + L * c;
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
            lw[j] = kNone;
            lu[j] = best;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (l + L * c < m) atomicMin(&lw[prop[c]], l + L * c);
    __builtin_amdgcn_wave_barrier();
    double th = lu[0];
    for (int j = 1; j < m; ++j) th = th + lu[j];
    unsigned long long unm = 0ull;  // rows left unmatched, group-uniform
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = l + L * c;
        if (j < m) p[c] = (lw[prop[c]] == j) ? prop[c] : -1;
        const unsigned long long b = __builtin_amdgcn_ballot_w64(j < m && lw[j] == kNone) & gmask;
        unm |= (b >> gbase) << (L * c);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = l + L * c;
        if (j < m) {
            lp[j] = p[c];
            lu[j] = 0.0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    int st = 0;
    int i0 = unm ? __builtin_ctzll(unm) : m, r = 0, last = -1;
    bool fresh = true;
    while (i0 < m) {
        if (fresh) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                minv[c] = kInf;
                way[c] = -1;
            }
            used = 0u;
            intree = (((unsigned)i0 % L) == (unsigned)l) ? (1u << ((unsigned)i0 / L)) : 0u;
            r = i0;
            last = -1;
            fresh = false;
        }
        ++st;
        const double ur = lu[r];
        const double *row = M + __umul24((unsigned)r, (unsigned)m);  // (r * m < 2^24: a full-rate multiply)
        double best = kInf;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m && !((used >> c) & 1u)) {
                const double s = (row[j] - ur) - v[c];
                if (s < minv[c]) {
                    minv[c] = s;
                    way[c] = last;
                }
                best = dmin(best, minv[c]);
            }
        }
        const double mn = group_min<L>(best);
        // chosen column: tied non-tree columns, unmatched first, lowest
        // index: each lane offers its lowest tied column (and its lowest
        // unmatched one), then the group takes the least of the offers
        int jf = kNone, ja = kNone;
#pragma unroll
        for (int c = C - 1; c >= 0; --c) {
            const int j = l + L * c;
            if (j < m && !((used >> c) & 1u) && minv[c] == mn) {
                ja = j;
                if (p[c] < 0) jf = j;
            }
        }
        jf = group_min_i32<L>(jf);
        ja = group_min_i32<L>(ja);
        const int js = (jf != kNone) ? jf : ja;
        const double delta = mn;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if ((intree >> c) & 1u) u[c] = u[c] + delta;
            if (j < m) {
                if ((used >> c) & 1u)
                    v[c] = v[c] - delta;
                else
                    minv[c] = minv[c] - delta;
            }
        }
        th = th + delta;
        const int pj = lp[js];
        if (pj < 0) {
            // Flip the alternating path js <- way[js] <- ... <- root: every
            // column on it takes the old row of its predecessor (the root row
            // i0 for the first column).  Tree rows publish their potentials.
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int j = l + L * c;
                if (j < m) lw[j] = way[c];
                if ((intree >> c) & 1u) lu[j] = u[c];
            }
            __builtin_amdgcn_wave_barrier();
            unsigned onpath = 0u;
            int j = js;
            while (j >= 0) {
                if (((unsigned)j % L) == (unsigned)l) onpath |= 1u << ((unsigned)j / L);
                j = lw[j];
            }
            int np[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int w = way[c];
                np[c] = (w < 0) ? i0 : lp[w < 0 ? 0 : w];
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if ((onpath >> c) & 1u) {
                    p[c] = np[c];
                    lp[l + L * c] = np[c];
                }
            }
            __builtin_amdgcn_wave_barrier();
            unm &= unm - 1ull;
            i0 = unm ? __builtin_ctzll(unm) : m;
            fresh = true;
        } else {
            // (js, pj >= 0: unsigned division by L is a mask and a shift)
            if (((unsigned)js % L) == (unsigned)l) used |= 1u << ((unsigned)js / L);
            if (((unsigned)pj % L) == (unsigned)l) intree |= 1u << ((unsigned)pj / L);
            r = pj;
            last = js;
        }
    }
    theta = th;
    steps = st;
}

}  // namespace qap
