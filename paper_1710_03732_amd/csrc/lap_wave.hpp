// lap_wave.hpp -- Hungarian LAP solver for one group of L lanes of a 64-wide
// CDNA wavefront (L in {8, 16, 32, 64}); lane l owns columns (and rows)
// l + L*c for c < C, so m <= L*C.
//
// The method: shortest augmenting paths with row/column potentials, the
// primal-dual Hungarian algorithm that solves every Z-, Y- and X-LAP of the
// three-stage decomposition of DLRLT2 (Section 2.3, "LAP Solution").  The
// paper does not say which optimal duals a solver must return; this solver
// makes the fixed choice the whole library is built on:
//   * cold start, rows inserted in order 0..m-1;
//   * a Dijkstra step scans the newest tree row r: every non-tree column j
//     computes s = (M[r][j] - u[r]) - v[j] and keeps it in minv[j] when
//     strictly smaller, remembering the column through which it was reached;
//   * the next column is the non-tree column of least minv; ties prefer an
//     unmatched column, then the lowest index;
//   * delta = that least minv; tree rows u += delta, tree columns v -= delta,
//     non-tree columns minv -= delta; the LAP value is the running sum of the
//     deltas;
//   * reaching an unmatched column flips the alternating path to the root.
// Every per-column operation is one IEEE add, subtract or compare, and the
// argmin is an exact min reduction, so the result does not depend on L or C.
//
// Per step the group does one LDS row read per slot, two subtracts, a
// butterfly min over the group (double) and one over an int code that
// encodes the tie-break, plus two broadcasts (row potential, matched row).
#pragma once
#include <hip/hip_runtime.h>

namespace qap {

constexpr double kInf = __builtin_huge_val();

template <int L>
__device__ __forceinline__ double group_min(double x)
{
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) {
        const double y = __shfl_xor(x, off, L);
        x = (y < x) ? y : x;
    }
    return x;
}

template <int L>
__device__ __forceinline__ int group_min(int x)
{
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) {
        const int y = __shfl_xor(x, off, L);
        x = (y < x) ? y : x;
    }
    return x;
}

template <int C, typename T>
__device__ __forceinline__ T slot(const T (&a)[C], int s)
{
    T r = a[0];
#pragma unroll
    for (int c = 1; c < C; ++c)
        if (s == c) r = a[c];
    return r;
}

// Solve the m x m LAP whose matrix row r starts at M + r*ld (LDS or global).
// Outputs per slot c (index j = l + L*c): u[c] = potential of row j, v[c] =
// potential of column j, p[c] = row assigned to column j (-1 if j >= m).
// theta = LAP value, steps = Dijkstra steps.  All lanes of the group must be
// active; other groups of the wave may be doing their own solve.
template <int L, int C>
__device__ void lap_solve(const double *__restrict__ M, int ld, int m, int l, double (&u)[C],
                          double (&v)[C], int (&p)[C], double &theta, int &steps)
{
    double minv[C];
    int way[C];
    unsigned used = 0u, intree = 0u;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        u[c] = 0.0;
        v[c] = 0.0;
        p[c] = -1;
        minv[c] = kInf;
        way[c] = -1;
    }
    double th = 0.0;
    int st = 0;
    int i0 = 0, r = 0, last = -1;
    bool fresh = true;
    while (i0 < m) {
        if (fresh) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                minv[c] = kInf;
                way[c] = -1;
            }
            used = 0u;
            intree = ((i0 % L) == l) ? (1u << (i0 / L)) : 0u;
            r = i0;
            last = -1;
            fresh = false;
        }
        ++st;
        const double ur = __shfl(slot<C>(u, r / L), r % L, L);
        const double *row = M + (size_t)r * ld;
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
                best = (minv[c] < best) ? minv[c] : best;
            }
        }
        const double mn = group_min<L>(best);
        int code = 1 << 20;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m && !((used >> c) & 1u) && minv[c] == mn) {
                const int cc = (p[c] < 0) ? j : (j + 256);
                code = (cc < code) ? cc : code;
            }
        }
        code = group_min<L>(code);
        const int js = code & 255;
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
        const int pj = __shfl(slot<C>(p, js / L), js % L, L);
        if (pj < 0) {
            // Flip the alternating path js <- way[js] <- ... <- root: every
            // column on it takes the old row of its predecessor (the root row
            // i0 for the first column).
            unsigned onpath = 0u;
            int j = js;
            while (j >= 0) {
                if ((j % L) == l) onpath |= 1u << (j / L);
                j = __shfl(slot<C>(way, j / L), j % L, L);
            }
            int np[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int w = way[c];
                const int ws = (w < 0) ? 0 : w;
                int got = 0;
#pragma unroll
                for (int cc = 0; cc < C; ++cc) {
                    const int val = __shfl(p[cc], ws % L, L);
                    if ((ws / L) == cc) got = val;
                }
                np[c] = (w < 0) ? i0 : got;
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                if ((onpath >> c) & 1u) p[c] = np[c];
            ++i0;
            fresh = true;
        } else {
            if ((js % L) == l) used |= 1u << (js / L);
            if ((pj % L) == l) intree |= 1u << (pj / L);
            r = pj;
            last = js;
        }
    }
    theta = th;
    steps = st;
}

}  // namespace qap
