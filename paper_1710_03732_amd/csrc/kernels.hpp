// kernels.hpp -- device kernels of one F1 RLT2 dual-ascent iteration
// (Algorithm 1 of Date & Nagi in the "fast" form of Section 3.4).
//
//   k_init        x/y/z costs of Section 2.1 (RLT1 C_ijpq = f_ij d_pq, no
//                 cubic terms), fill kernels instead of memsets
//   k_sweep       Type 1-3 ascent rules (Eqs. da:rule1-3) combined as in the
//                 proof of Theorem 1 (Eqs. ch4:proof:2-4), one thread per
//                 orbit of six symmetric z variables (Eq. rlt2:con3)
//   k_scale_xy    the x and y levels keep (1-kappa) of their slack
//   k_zlap        Z-LAPs (Theta_ijpq, xi, psi), one lane group per tile
//   k_ylap_s      y-pair rule (Eq. da:yrule1) fused into the load, then the
//                 Y-LAPs (Delta_ip, gamma, delta)
//   k_xlap        the X-LAP, bound, incumbent, feasibility check, stop flag
//
// Device layout (see include/qap_rlt2.h): tiles t(i,p,j,q) =
// ((i*n+p)*(n-1)+j')*(n-1)+q'; z entries tile-major with compressed row k''
// and column r''.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lap_scalar.hpp"
#include "lap_wave.hpp"

namespace qap {

constexpr int kStepBins = 4096;  // Dijkstra-step counters, spread to avoid atomic contention

struct DevScalars {
    double lb;
    double ub;
    int t;             // iterations completed
    int proven;
    int integer_data;
    int stopped;       // set once the bound proves optimality or gap < min_gap
    int reason;        // why a batched node stopped (1 fathomed, 2 window rule, 3 gap)
    int sa_steps;      // Type 4 steps taken
    unsigned long long steps;
    double best;       // best bound of any iteration (a Type 4 step lowers lb)
};

struct SweepConsts {
    double kz, okz, ky2, kx3, phi;
    double phil;  // HALF: share of a lower member's g for each upper partner
};

// Tile index of the ordered pair ((f1,l1),(f2,l2)), f1 != f2, l1 != l2.
__device__ __forceinline__ long long tile_of(int n, int f1, int l1, int f2, int l2)
{
    const int f2p = f2 - (f2 > f1);
    const int l2p = l2 - (l2 > l1);
    return ((long long)(f1 * n + l1) * (n - 1) + f2p) * (n - 1) + l2p;
}

// Tile index of the b-th tile (i,p,j,q) with i < j, in ascending tile order
// (the tiles the HALF scheme solves).  Facility i owns n (n-1-i) (n-1) of
// them (any p, j' >= i, any q').  b < n^2 (n-1)^2 / 2 fits 32 bits; the loop
// and the divisions are wave-uniform.
__device__ __forceinline__ long long upper_tile(unsigned b, int n)
{
    const unsigned n1 = (unsigned)n - 1u;
    unsigned i = 0u, per = (unsigned)n * n1 * n1;
    while (b >= per) {
        b -= per;
        ++i;
        per = (unsigned)n * (n1 - i) * n1;
    }
    const unsigned row = (n1 - i) * n1;  // tiles per (i, p)
    const unsigned p = b / row, r2 = b % row;
    const unsigned jp = i + r2 / n1, qp = r2 % n1;
    return (((long long)i * n + p) * n1 + jp) * n1 + qp;
}

// Copies count doubles from global src to LDS dst with the nthr threads
// numbered tid.  Each thread issues a batch of kBatch loads before any of
// their LDS writes, so it waits for HBM once per batch.  (A plain strided
// loop with a run-time trip count compiles to load, wait, write per element:
// one full memory latency per element.)
template <int kBatch = 16>
__device__ __forceinline__ void copy_to_lds(double *__restrict__ dst, const double *__restrict__ src, int count,
                                            int tid, int nthr)
{
    for (int base = 0; base < count; base += kBatch * nthr) {
        double buf[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int e = base + tid + nthr * k;
            if (e < count) buf[k] = src[e];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int e = base + tid + nthr * k;
            if (e < count) dst[e] = buf[k];
        }
    }
}

// ------------------------------------------------------------------ init --
__global__ void k_fill(double *__restrict__ a, size_t count, double val)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) a[i] = val;
}

__global__ void k_init_xy(const double *__restrict__ F, const double *__restrict__ D,
                          const double *__restrict__ B, double *__restrict__ Xc,
                          double *__restrict__ Yc, int n)
{
    const long long T = (long long)n * n * (n - 1) * (n - 1);
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < T; e += stride) {
        const int m1 = n - 1;
        const int qp = (int)(e % m1);
        const int jp = (int)((e / m1) % m1);
        const int ip = (int)(e / ((long long)m1 * m1));
        const int i = ip / n, p = ip % n;
        const int j = jp + (jp >= i), q = qp + (qp >= p);
        Yc[e] = F[i * n + j] * D[p * n + q];
    }
    e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < (long long)n * n; e += stride) {
        const int i = (int)(e / n), p = (int)(e % n);
        Xc[e] = B[e] + F[i * n + i] * D[p * n + p];
    }
}

// ----------------------------------------------------------------- sweep --
// Orbit {A=(i,p), B=(j,q), C=(k,r)}, i<j<k.  Members in canonical order
// (A,B,C),(A,C,B),(B,A,C),(B,C,A),(C,A,B),(C,B,A); member (P1,P2,P3) is the z
// entry in tile (P1,P2) at row P3.fac, column P3.loc; its y parent is that
// tile and its x parent P1.  The z array holds pi_z of the last Z-LAPs:
//   g_e   = (kz*pi_z(e) + ky2*pi_y(tile(e))) + kx3*pi_x(P1(e))
//   new_e = okz*pi_z(e) + phi*(left fold of g_f over f != e, canonical order)
//
// For one facility triple the six members form six axis-permuted copies of a
// 3-D array over the locations (p,q,r): member e is contiguous along its
// third location.  A block takes one triple and one CB^3 cube of locations
// and transposes through LDS: load phase (each member read as runs of CB
// contiguous doubles along its own last axis, pi_z staged in a padded
// [p][q][r] layout, pi_y / pi_x of the block's tiles and pairs read once),
// orbit phase (one thread per orbit forms the six g and the shares), store
// phase (runs again).  Block numbering keeps all cubes of one triple on one
// XCD, back to back, so the partial cache lines at run ends merge in that
// XCD's L2.
constexpr int SB = 8;                       // cube edge of the warm-start writer and batched sweep
constexpr int SB_Q = SB + 1;                // padded q pitch
constexpr int SB_P = SB * SB_Q + 1;         // padded p pitch
constexpr int SB_CUBE = SB * SB_P;          // doubles per staged member

__device__ __forceinline__ int cube_idx(int pl, int ql, int rl) { return pl * SB_P + ql * SB_Q + rl; }

// The ascent sweep's cube, edge CB chosen per n (8, or 10 where its cubes
// leave fewer slots outside the instance): padded LDS pitches, one thread
// per orbit, whole waves.
template <int CB>
struct Cube {
    static constexpr int Q = CB + 1;                 // padded q pitch
    static constexpr int P = CB * Q + 1;             // padded p pitch
    static constexpr int SIZE = CB * P;              // doubles per staged member
    static constexpr int ORB = CB * CB * CB;         // orbits per block
    static constexpr int NT = (ORB + 63) / 64 * 64;  // threads per block
    __device__ static __forceinline__ int idx(int pl, int ql, int rl) { return pl * P + ql * Q + rl; }
};

//
// With TRACK the sweep also accumulates each entry's Lagrange multiplier
// change, g_e - phi * sum_{f != e} g_f (its own shares minus what it
// receives from its partners, Eq. ch4:proof:2), into Vt (same layout as Z).
//
// HALF (Section 5): only the upper members, whose first two facilities
// ascend (canonical positions 0, 1, 3), hold z entries; the lower ones
// (2, 4, 5) sit in unsolved tiles and stay 0, so they are neither read nor
// written.  A lower member's g is its y and x shares alone (its z value is
// 0), and
//   new_e = okz*pi_z(e) + (phi*(g of the two upper partners, canonical order)
//                          + phil*((g_2 + g_4) + g_5))   for e in {0, 1, 3}.
//
// POOL is the two-phase variant's pooling between its two Z-LAP solves
// (Section 3.4), on the same transpose: the orbit phase splits the six
// slacks into S_N (> 0) and S_B (<= 0); when both are non-empty the S_N
// members become 0 and each S_B member gains (left fold of the S_N slacks,
// canonical order) / |S_B|.  No y or x duals are involved.
//
// SLOW (with TRACK) is the slow variant's sweep: the tracked multiplier
// moves as above and z is rebuilt as its S-form cost, -v (D = 0), for LAPs
// on the full costs.  POOL with TRACK is S2's pooling: a changed entry's
// multiplier moves by its old slack minus its new one.
template <int CB, bool TRACK, bool HALF, bool POOL = false, bool SLOW = false>
__global__ __launch_bounds__(Cube<CB>::NT) void k_sweep(double *__restrict__ Z, const double *__restrict__ Py,
                                               const double *__restrict__ Px,
                                               const int *__restrict__ triples, int ntriples, int n,
                                               int nb, SweepConsts K, const DevScalars *__restrict__ S,
                                               double *__restrict__ Vt)
{
    if (S->stopped) return;
    // g_e staged per orbit position; the orbit phase overwrites it with phi*sum
    using C = Cube<CB>;
    __shared__ double gs[6 * C::SIZE];
    const unsigned b = blockIdx.x;
    const unsigned xcd = b & 7u, s = b >> 3;
    const unsigned nb3 = (unsigned)(nb * nb * nb);
    const int tri = (int)((s / nb3) * 8u + xcd);
    if (tri >= ntriples) return;
    const int sub = (int)(s % nb3);
    const int base[3] = {(sub / (nb * nb)) * CB, ((sub / nb) % nb) * CB, (sub % nb) * CB};
    const int packed = triples[tri];
    const int fi = packed & 0xff, fj = (packed >> 8) & 0xff, fk = (packed >> 16) & 0xff;
    const int m = n - 2;
    const long long mm = (long long)m * m;
    const int F1[6] = {fi, fi, fj, fj, fk, fk};
    const int F2[6] = {fj, fk, fi, fk, fi, fj};
    const int F3[6] = {fk, fj, fk, fi, fj, fi};
    const int X1[6] = {0, 0, 1, 1, 2, 2};
    const int X2[6] = {1, 2, 0, 2, 0, 1};
    const int X3[6] = {2, 1, 2, 0, 1, 0};
    constexpr int NT = C::NT;
    // pi_y of the block's tiles and pi_x of its (facility, location) pairs,
    // read once per block: member e's tile is fixed by its first two cube
    // coordinates (a1 along axis X1[e], a2 along X2[e]), its x parent by the
    // first.  Entries outside the instance hold 0 and are never used.  They
    // are loaded into registers here and written to LDS after the z loads
    // below have been issued, so the block waits for all of them at once.
    __shared__ double pys[6 * CB * CB];
    __shared__ double pxs[3 * CB];
    constexpr int YREP = POOL ? 0 : (6 * CB * CB + NT - 1) / NT;
    double yv[YREP > 0 ? YREP : 1];
    double xv = 0.0;
#pragma unroll
    for (int rep = 0; rep < YREP; ++rep) {
        const int a = threadIdx.x + NT * rep;
        yv[rep] = 0.0;
        if (a < 6 * CB * CB) {
            const int e = a / (CB * CB), a1 = (a / CB) % CB, a2 = a % CB;
            const int x1 = e >> 1, x2 = (0x102021 >> (4 * e)) & 0xf;  // X1[e], X2[e]
            const int f1 = x1 == 0 ? fi : (x1 == 1 ? fj : fk), f2 = x2 == 0 ? fi : (x2 == 1 ? fj : fk);
            const int l1 = (x1 == 0 ? base[0] : (x1 == 1 ? base[1] : base[2])) + a1;
            const int l2 = (x2 == 0 ? base[0] : (x2 == 1 ? base[1] : base[2])) + a2;
            yv[rep] = (l1 < n && l2 < n && l1 != l2) ? Py[tile_of(n, f1, l1, f2, l2)] : 0.0;
        }
    }
    if (!POOL && threadIdx.x < 3 * CB) {
        const int x = threadIdx.x / CB, l = (x == 0 ? base[0] : (x == 1 ? base[1] : base[2])) + threadIdx.x % CB;
        const int f = x == 0 ? fi : (x == 1 ? fj : fk);
        xv = l < n ? Px[f * n + l] : 0.0;
    }
    constexpr int PER = 1;  // one orbit per thread
    long long za[6][PER];
    int li[6][PER];
    bool ok[6][PER];
    double pz[6][PER];
    double pv[6][PER];  // TRACK: the entries' multipliers, read with pi_z
    // this thread's member-major elements (runs along each member's own last
    // location axis); pi_z goes to the cube for the orbit phase.  Thread
    // tid < CB^3 takes cube coordinates (a1, a2, a3) = (tid / CB^2,
    // tid / CB % CB, tid % CB); with CB = 8 a1 is the same for the whole
    // wave, so the tile row (f1, l1, f2) and the z row are a scalar offset.
    // Only l2' * m^2 + col always varies across the lanes (a 24-bit product).
    const bool live = (int)threadIdx.x < C::ORB;
    const int a1w = (CB * CB == 64) ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))
                                    : (int)threadIdx.x / (CB * CB);
    const int a2 = ((int)threadIdx.x / CB) % CB, a3 = (int)threadIdx.x % CB;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        if (HALF && (e == 2 || e == 4 || e == 5)) continue;
#pragma unroll
        for (int w = 0; w < PER; ++w) {
            const int a1 = a1w;
            int loc[3];
            loc[X1[e]] = base[X1[e]] + a1;
            loc[X2[e]] = base[X2[e]] + a2;
            loc[X3[e]] = base[X3[e]] + a3;
            const int l1 = loc[X1[e]], l2 = loc[X2[e]], l3 = loc[X3[e]];
            const bool v = live && l1 < n && l2 < n && l3 < n && l1 != l2 && l1 != l3 && l2 != l3;
            const int f1 = F1[e], f2 = F2[e], f3 = F3[e];
            const int f2p = f2 - (f2 > f1);
            const int row = f3 - (f3 > f1) - (f3 > f2);
            const long long zrow = ((long long)(f1 * n + l1) * (n - 1) + f2p) * (n - 1) * mm + (long long)row * m;
            const int l2p = l2 - (l2 > l1);
            const int col = l3 - (l3 > l1) - (l3 > l2);
            ok[e][w] = v;
            za[e][w] = v ? zrow + (long long)(__umul24((unsigned)l2p, (unsigned)mm) + col) : 0;
            li[e][w] = C::idx(loc[0] - base[0], loc[1] - base[1], loc[2] - base[2]);
            pz[e][w] = Z[za[e][w]];
            if constexpr (TRACK) pv[e][w] = Vt[za[e][w]];
        }
    }
#pragma unroll
    for (int rep = 0; rep < YREP; ++rep) {
        const int a = threadIdx.x + NT * rep;
        if (a < 6 * CB * CB) pys[a] = yv[rep];
    }
    if (!POOL && threadIdx.x < 3 * CB) pxs[threadIdx.x] = xv;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        if (HALF && (e == 2 || e == 4 || e == 5)) continue;
#pragma unroll
        for (int w = 0; w < PER; ++w)
            if (ok[e][w]) gs[e * C::SIZE + li[e][w]] = pz[e][w];
    }
    __syncthreads();
    // orbit phase: g of the six members, then phi * (left fold of the
    // partners' g), canonical order
#pragma unroll
    for (int w = 0; w < PER; ++w) {
        const int u = threadIdx.x + NT * w;
        const int rl = u % CB, ql = (u / CB) % CB, pl = u / (CB * CB);
        const int p = base[0] + pl, q = base[1] + ql, r = base[2] + rl;
        if (u < C::ORB && p < n && q < n && r < n && p != q && p != r && q != r) {
            const int c = C::idx(pl, ql, rl);
            if (POOL) {
                double v[6], slack = 0.0;
                int nbasic = 0;
                bool first = true;
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    v[e] = gs[e * C::SIZE + c];
                    if (v[e] > 0.0) {
                        slack = first ? v[e] : slack + v[e];
                        first = false;
                    } else {
                        ++nbasic;
                    }
                }
                if (nbasic != 0 && nbasic != 6) {
                    const double share = slack / (double)nbasic;
#pragma unroll
                    for (int e = 0; e < 6; ++e) gs[e * C::SIZE + c] = v[e] > 0.0 ? 0.0 : v[e] + share;
                }
                continue;
            }
            const int lc[3] = {pl, ql, rl};
            double g[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const double y = pys[(e * CB + lc[X1[e]]) * CB + lc[X2[e]]];
                const double x = pxs[X1[e] * CB + lc[X1[e]]];
                if (HALF && (e == 2 || e == 4 || e == 5))
                    g[e] = (1.0 * 0.0 + K.ky2 * y) + K.kx3 * x;
                else
                    g[e] = (K.kz * gs[e * C::SIZE + c] + K.ky2 * y) + K.kx3 * x;
            }
            if (HALF) {
                const double low = K.phil * ((g[2] + g[4]) + g[5]);
                gs[0 * C::SIZE + c] = K.phi * (g[1] + g[3]) + low;
                gs[1 * C::SIZE + c] = K.phi * (g[0] + g[3]) + low;
                gs[3 * C::SIZE + c] = K.phi * (g[0] + g[1]) + low;
                continue;
            }
            gs[0 * C::SIZE + c] = K.phi * ((((g[1] + g[2]) + g[3]) + g[4]) + g[5]);
            gs[1 * C::SIZE + c] = K.phi * ((((g[0] + g[2]) + g[3]) + g[4]) + g[5]);
            gs[2 * C::SIZE + c] = K.phi * ((((g[0] + g[1]) + g[3]) + g[4]) + g[5]);
            gs[3 * C::SIZE + c] = K.phi * ((((g[0] + g[1]) + g[2]) + g[4]) + g[5]);
            gs[4 * C::SIZE + c] = K.phi * ((((g[0] + g[1]) + g[2]) + g[3]) + g[5]);
            gs[5 * C::SIZE + c] = K.phi * ((((g[0] + g[1]) + g[2]) + g[3]) + g[4]);
        }
    }
    __syncthreads();
    // store phase, back along the same runs.  Every output is formed first,
    // each in registers of its own (the empty asm keeps it out of its store's
    // branch), then the stores: formed inside the branches, each value's wait
    // for its loads also counted the stores issued before it, so the later
    // stores waited for the earlier ones to complete.
    //   plain:  new_e = okz*pi_z(e) + phi*sum
    //   POOL:   the pooled value, stored only where its bits changed (most
    //           orbits have no zero slack among the six and stay as they are)
    //   TRACK:  v_e += g_e - phi*sum; with POOL, v_e += old slack - new slack
    //   SLOW:   z_e = -v_e (the S-form cost of the tracked multiplier)
    double zo[6][PER], vo[6][PER];
    bool so[6][PER];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        if (HALF && (e == 2 || e == 4 || e == 5)) continue;
#pragma unroll
        for (int w = 0; w < PER; ++w) {
            const double share = gs[e * C::SIZE + li[e][w]];
            so[e][w] = ok[e][w] && !(POOL && __double_as_longlong(share) == __double_as_longlong(pz[e][w]));
            double v = 0.0;
            if constexpr (TRACK && POOL) {
                v = pv[e][w] + (pz[e][w] - share);
            } else if constexpr (TRACK) {
                const int u = threadIdx.x + NT * w;
                const int a2 = (u / CB) % CB, a1 = u / (CB * CB);
                const double y = pys[(e * CB + a1) * CB + a2];
                const double x = pxs[X1[e] * CB + a1];
                const double g = (K.kz * pz[e][w] + K.ky2 * y) + K.kx3 * x;
                v = pv[e][w] + (g - share);
            }
            zo[e][w] = SLOW ? -v : (POOL ? share : K.okz * pz[e][w] + share);
            vo[e][w] = v;
            asm volatile("" : "+v"(zo[e][w]));
            if constexpr (TRACK) asm volatile("" : "+v"(vo[e][w]));
        }
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        if (HALF && (e == 2 || e == 4 || e == 5)) continue;
#pragma unroll
        for (int w = 0; w < PER; ++w)
            if (so[e][w]) {
                Z[za[e][w]] = zo[e][w];
                if constexpr (TRACK) Vt[za[e][w]] = vo[e][w];
            }
    }
}

// Slow variant: after its sweep the x and y levels restart from the full
// costs, b + f_ii d_pp and f_ij d_pq (the y multipliers stay 0), and the
// bound from 0, so the X-LAP gives the whole bound of the new multipliers.
__global__ void k_slow_reset(const double *__restrict__ F, const double *__restrict__ D,
                             const double *__restrict__ B, double *__restrict__ Xc, double *__restrict__ Yc,
                             int n, DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    const long long T = (long long)n * n * (n - 1) * (n - 1);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < T; e += stride) {
        const int m1 = n - 1;
        const int qp = (int)(e % m1);
        const int jp = (int)((e / m1) % m1);
        const int ip = (int)(e / ((long long)m1 * m1));
        const int i = ip / n, p = ip % n;
        const int j = jp + (jp >= i), q = qp + (qp >= p);
        Yc[e] = F[i * n + j] * D[p * n + q];
    }
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)n * n; e += stride) {
        const int i = (int)(e / n), p = (int)(e % n);
        Xc[e] = B[e] + F[i * n + i] * D[p * n + p];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) S->lb = 0.0;
}

// R_y <- (1-ky) pi_y, R_x <- (1-kx) pi_x (after the sweep has read them).
__global__ void k_scale_xy(double *__restrict__ Yc, const double *__restrict__ Py,
                           double *__restrict__ Xc, const double *__restrict__ Px, long long T,
                           int nn, double oky, double okx, const DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long a = e; a < T; a += stride) Yc[a] = oky * Py[a];
    for (long long a = e; a < nn; a += stride) Xc[a] = okx * Px[a];
}

// ----------------------------------------------------------------- Z-LAP --
// Groups of L lanes, G = blockDim/L groups per block.  LDS: the G tiles
// (contiguous, filled by one coalesced copy of G consecutive tiles) followed
// by G scratch areas of 2m doubles (potentials, matching, path links).  After
// the solve each tile's slacks pi_z = (M - u_row) - v_col go back to HBM in
// place, again as one coalesced pass, and Theta is added to R_y.
template <int L, int C>
__global__ __launch_bounds__(256) void k_zlap(double *__restrict__ Z, double *__restrict__ Yc, int m,
                                              long long T, DevScalars *__restrict__ S,
                                              unsigned long long *__restrict__ bins)
{
    if (S->stopped) return;
    extern __shared__ double lds[];
    __shared__ unsigned long long bsteps;
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const int gbase = (threadIdx.x & 63) - l;
    const long long t0 = (long long)blockIdx.x * G;
    const int mm = m * m;
    const long long left = T - t0;
    const int nt = (int)(left < G ? left : G);
    double *src = Z + t0 * mm;
    copy_to_lds(lds, src, nt * mm, threadIdx.x, blockDim.x);
    const long long t = t0 + g;
    const double yc0 = (g < nt) ? Yc[t] : 0.0;  // read now, added to after the solve
    double *scr = lds + (size_t)G * mm + (size_t)g * 2 * m;
    double *lu = scr;
    int *lp = (int *)(scr + m);
    int *lw = lp + m;
    if (threadIdx.x == 0) bsteps = 0ull;
    __syncthreads();
    int st = 0;
    if (g < nt) {
        double u[C], v[C], th;
        int pc[C];
        lap_solve<L, C>(lds + (size_t)g * mm, m, l, gbase, lu, lp, lw, u, v, pc, th, st);
        __builtin_amdgcn_wave_barrier();
        double *vs = scr + m;  // column potentials over the matching/links area
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m) vs[j] = v[c];
        }
        if (l == 0) {
            Yc[t] = yc0 + th;
            atomicAdd(&bsteps, (unsigned long long)st);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * mm; e += blockDim.x) {
        const int gg = e / mm, w = e - gg * mm;
        const double *us = lds + (size_t)G * mm + (size_t)gg * 2 * m;
        src[e] = (lds[e] - us[w / m]) - us[m + w % m];
    }
    if (threadIdx.x == 0) atomicAdd(&bins[blockIdx.x & (kStepBins - 1)], bsteps);
}

// Z-LAPs with the scalar-controlled solver: one wavefront per block holding
// H tiles (H = 2: two 32-lane LAPs, m <= 32; H = 1: one 64-lane LAP).
// MC > 0 compiles the kernel for tiles of size MC (m must equal it): the
// tile copy, the column reduction and the write-back then run with constant
// trip counts and immediate offsets.  Same arithmetic in the same order.
// KR > 0 (one LAP of a fixed size): the tile's first KR rows go to registers
// rather than LDS (see lap_solve_scalar1), so a LAP takes KR*m*8 bytes less
// LDS and more of them are resident on a CU.
template <int H, int MC = 0, int KR = 0>
__global__ __launch_bounds__(64) void k_zlap_s(double *__restrict__ Z, double *__restrict__ Yc, int m_in,
                                               long long T, DevScalars *__restrict__ S,
                                               unsigned long long *__restrict__ bins, int half)
{
    static_assert(KR == 0 || (H == 1 && MC >= KR && KR <= 24), "register rows need one LAP of a fixed size");
    if (S->stopped) return;
    extern __shared__ double lds[];
    constexpr int W = 64 / H;
    const int m = MC > 0 ? MC : m_in;
    const int lane = (int)(threadIdx.x & 63);  // (the mask tells the compiler lane < 64)
    const int h = (H == 1) ? 0 : (lane >> 5);
    const int l = lane & (W - 1);
    // HALF (H = 1): block b solves the b-th tile with i < j
    const long long t0 = (H == 1 && half) ? upper_tile(blockIdx.x, m + 2) : (long long)blockIdx.x * H;
    const int mm = m * m;
    const long long left = T - t0;
    // (one tile per block: every block of the grid has its tile)
    const int nt = (H == 1) ? 1 : (int)(left < H ? left : H);
    double *src = Z + t0 * mm;
    dreg16 R = {};
    dreg8 R2 = {};
    if constexpr (KR > 0) {
        const int cl = lane < m ? lane : 0;  // lanes past m hold a copy of column 0 (never used)
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            if (r < 16)
                R[r] = src[r * m + cl];
            else
                R2[r - 16] = src[r * m + cl];
        }
    }
    copy_to_lds(lds, src + KR * m, nt * mm - KR * m, lane, 64);
    const double yc0 = (h < nt) ? Yc[t0 + h] : 0.0;  // read now, added to after the solve
    double *scr = lds + (size_t)H * mm - KR * m;
    int toff[H], soff[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int qq = q < nt ? q : 0;
        toff[q] = qq * mm;
        soff[q] = H * mm - KR * m + qq * 2 * m;
    }
    __syncthreads();
    double u, v, th;
    int p, st;
    if constexpr (H == 1) {
        if (KR == 0 && m <= 16)
            lap_solve_scalar1<16, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
        else if (m <= 32)
            lap_solve_scalar1<32, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
        else
            lap_solve_scalar1<64, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
    } else {
        if (m <= 16)
            lap_solve_scalar2<16>(lds, toff, soff, m, nt, u, v, p, th, st);
        else
            lap_solve_scalar2<32>(lds, toff, soff, m, nt, u, v, p, th, st);
    }
    __builtin_amdgcn_wave_barrier();
    // v to the scratch after the potentials (matching and links are done);
    // with one LAP per wave (whose scratch has no room for v) it is fetched
    // from its lane instead
    if (H == 2 && l < m && h < nt) scr[(size_t)h * 2 * m + m + l] = v;
    __syncthreads();
    // slacks back in place, row by row (no index division): a lane owns one
    // column; with one LAP of m <= 32 per wave the two half-waves take
    // alternate rows
    {
        const bool two = (H == 1) && (m <= 32);
        const int sub = two ? (lane >> 5) : 0;
        const int col = (H == 1 && !two) ? lane : (lane & 31);
        const double vcol = (H == 1) ? __shfl(v, col) : 0.0;  // every lane takes part
        const double *us = scr + (size_t)h * 2 * m;
        double *dst = src + (size_t)h * mm;
        if constexpr (KR > 0) {
            // the register rows: lane l holds column l and its v
            if (lane < m) {
#pragma unroll
                for (int r = 0; r < KR; ++r) dst[r * m + lane] = ((r < 16 ? R[r] : R2[r - 16]) - us[r]) - v;
            }
        }
        if (h < nt && col < m) {
            const double vc = (H == 1) ? vcol : us[m + col];
            const double *tl = lds + (size_t)h * mm - KR * m;  // row r >= KR at tl + r*m
            const int step = two ? 2 : 1;
            // a constant trip count (rows past m skipped) lets a fixed m unroll it
            for (int k = 0; k < (m - KR + step - 1) / step; ++k) {
                const int r = KR + k * step + sub;
                if (r < m) dst[r * m + col] = (tl[r * m + col] - us[r]) - vc;
            }
        }
    }
    if (l == 0 && h < nt) Yc[t0 + h] = yc0 + th;
    int stt = st;
    if (H == 2) stt = __builtin_amdgcn_readlane(st, 0) + (nt > 1 ? __builtin_amdgcn_readlane(st, 32) : 0);
    if (lane == 0) atomicAdd(&bins[blockIdx.x & (kStepBins - 1)], (unsigned long long)stt);
}

// LAP batch with the scalar-controlled solver (validation entry point);
// MC > 0 and KR > 0 as for k_zlap_s.
template <int H, int MC = 0, int KR = 0>
__global__ __launch_bounds__(64) void k_lap_batch_s(const double *__restrict__ cost, int count, int m_in,
                                                    double *__restrict__ uo, double *__restrict__ vo,
                                                    double *__restrict__ tho, int *__restrict__ rco)
{
    static_assert(KR == 0 || (H == 1 && MC >= KR && KR <= 24), "register rows need one LAP of a fixed size");
    extern __shared__ double lds[];
    constexpr int W = 64 / H;
    const int m = MC > 0 ? MC : m_in;
    const int lane = (int)(threadIdx.x & 63);
    const int h = (H == 1) ? 0 : (lane >> 5);
    const int l = lane & (W - 1);
    const long long t0 = (long long)blockIdx.x * H;
    const int mm = m * m;
    const long long left = count - t0;
    const int nt = (int)(left < H ? left : H);
    const double *src = cost + t0 * mm;
    dreg16 R = {};
    dreg8 R2 = {};
    if constexpr (KR > 0) {
        const int cl = lane < m ? lane : 0;
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            if (r < 16)
                R[r] = src[r * m + cl];
            else
                R2[r - 16] = src[r * m + cl];
        }
    }
    copy_to_lds(lds, src + KR * m, nt * mm - KR * m, lane, 64);
    int toff[H], soff[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int qq = q < nt ? q : 0;
        toff[q] = qq * mm;
        soff[q] = H * mm - KR * m + qq * 2 * m;
    }
    __syncthreads();
    double u, v, th;
    int p, st;
    if constexpr (H == 1) {
        if (KR == 0 && m <= 16)
            lap_solve_scalar1<16, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
        else if (m <= 32)
            lap_solve_scalar1<32, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
        else
            lap_solve_scalar1<64, KR>(lds, toff[0], soff[0], m, u, v, p, th, st, R, R2);
    } else {
        if (m <= 16)
            lap_solve_scalar2<16>(lds, toff, soff, m, nt, u, v, p, th, st);
        else
            lap_solve_scalar2<32>(lds, toff, soff, m, nt, u, v, p, th, st);
    }
    if (l < m && h < nt) {
        const long long t = t0 + h;
        uo[t * m + l] = u;
        vo[t * m + l] = v;
        rco[t * m + l] = p;
        if (l == 0) tho[t] = th;
    }
}

// ----------------------------------------------------------------- Y-LAP --
// One Y-LAP per (i,p); its (n-1)x(n-1) block of R_y is contiguous.  For
// t >= 1 every entry is first replaced by ophy*R_y[ijpq] + phy*R_y[jiqp]
// (the y-pair rule applied by both members of the pair).  Writes pi_y to Py
// and adds Delta_ip to R_x.  With Ut (same layout as Yc) each entry's
// multiplier moves by phy * (own - partner) (Eq. da:yrule1).
//
// One wavefront per Y-LAP (i,p) with the scalar-controlled solver.  A Y-LAP
// phase has only n^2 LAPs, one or a few per SIMD: what counts is how fast one
// LAP is solved, and a step of this solver is the shortest (a lane-group
// mapping took 2.6 times as long at n = 30).
__global__ __launch_bounds__(64) void k_ylap_s(const double *__restrict__ Yc, double *__restrict__ Py,
                                               double *__restrict__ Xc, int n, int equalize, double ophy,
                                               double phy, DevScalars *__restrict__ S,
                                               unsigned long long *__restrict__ bins, double *__restrict__ Ut)
{
    if (S->stopped) return;
    extern __shared__ double lds[];
    const int lane = (int)(threadIdx.x & 63);
    const int m = n - 1, mm = m * m;
    const int ip = blockIdx.x;
    const int i = ip / n, p = ip % n;
    const long long base = (long long)ip * mm;
    const double xc0 = Xc[ip];  // read now, added to after the solve
    for (int e0 = 0; e0 < mm; e0 += 8 * 64) {
        double av[8], bv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + lane + 64 * k;
            if (e < mm) {
                av[k] = Yc[base + e];
                if (equalize) {
                    const int jp = e / m, qp = e % m;
                    const int j = jp + (jp >= i), q = qp + (qp >= p);
                    bv[k] = Yc[((long long)(j * n + q) * m + (i - (i > j))) * m + (p - (p > q))];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + lane + 64 * k;
            if (e < mm) {
                double a = av[k];
                if (equalize) {
                    const double b = bv[k];
                    if (Ut) Ut[base + e] = Ut[base + e] + phy * (a - b);
                    a = ophy * a + phy * b;
                }
                lds[e] = a;
            }
        }
    }
    __syncthreads();
    double u, v, th;
    int pc, st;
    if (m <= 16)
        lap_solve_scalar1<16>(lds, 0, mm, m, u, v, pc, th, st);
    else if (m <= 32)
        lap_solve_scalar1<32>(lds, 0, mm, m, u, v, pc, th, st);
    else
        lap_solve_scalar1<64>(lds, 0, mm, m, u, v, pc, th, st);
    __builtin_amdgcn_wave_barrier();
    // slacks out row by row (the scratch holds the row potentials); with
    // m <= 32 the two half-waves take alternate rows
    const bool two = m <= 32;
    const int sub = two ? (lane >> 5) : 0, col = two ? (lane & 31) : lane;
    const double vc = __shfl(v, col);  // every lane takes part
    if (col < m) {
        const double *us = lds + mm;
        const int step = two ? 2 : 1;
        for (int r = sub; r < m; r += step) Py[base + r * m + col] = (lds[r * m + col] - us[r]) - vc;
    }
    if (lane == 0) {
        Xc[ip] = xc0 + th;
        atomicAdd(&bins[blockIdx.x & (kStepBins - 1)], (unsigned long long)st);
    }
}

// ----------------------------------------------------------------- X-LAP --
// One wave (scalar-controlled solver).  LB += theta_x; pi_x -> Px;
// alpha/beta; the assignment is a QAP
// solution whose exact cost (int64 for integer data) updates the incumbent;
// feasibility check and gap test set the stop flag.
__global__ __launch_bounds__(64) void k_xlap(const double *__restrict__ Xc, double *__restrict__ Px,
                                             double *__restrict__ alpha, double *__restrict__ beta,
                                             const double *__restrict__ F, const double *__restrict__ D,
                                             const double *__restrict__ B, int *__restrict__ xperm,
                                             int *__restrict__ bestperm, double *__restrict__ trace,
                                             int n, double min_gap, double offset,
                                             DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    // the cost matrix, then the solver's scratch (row potentials, one int
    // per column)
    __shared__ double M[64 * 64 + 64 + 32];
    __shared__ double vs[64];
    __shared__ int sig[64];
    __shared__ int improved;
    const int l = threadIdx.x;
    const int nn = n * n;
    copy_to_lds(M, Xc, nn, l, 64);
    __syncthreads();
    double u, v, th;
    int pc, st;
    if (n <= 16)
        lap_solve_scalar1<16>(M, 0, nn, n, u, v, pc, th, st);
    else if (n <= 32)
        lap_solve_scalar1<32>(M, 0, nn, n, u, v, pc, th, st);
    else
        lap_solve_scalar1<64>(M, 0, nn, n, u, v, pc, th, st);
    if (l < n) {
        vs[l] = v;
        alpha[l] = u;
        beta[l] = v;
        sig[pc] = l;
    }
    __syncthreads();
    const double *lu = M + nn;  // the row potentials
    for (int e = l; e < nn; e += 64) Px[e] = (M[e] - lu[e / n]) - vs[e % n];
    // exact cost of the assignment
    double cd = 0.0;
    long long ci = 0;
    const int integer_data = S->integer_data;
    if (l < n) {
        const int si = sig[l];
        if (integer_data) {
            ci = (long long)B[l * n + si];
            for (int jj = 0; jj < n; ++jj)
                ci += (long long)F[l * n + jj] * (long long)D[si * n + sig[jj]];
        } else {
            cd = B[l * n + si];
            for (int jj = 0; jj < n; ++jj) cd = cd + F[l * n + jj] * D[si * n + sig[jj]];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ci += __shfl_xor(ci, off, 64);
        cd += __shfl_xor(cd, off, 64);
    }
    if (l == 0) {
        const double cost = (integer_data ? (double)ci : cd) + offset;
        const double lb = S->lb + th;
        S->lb = lb;
        double ub = S->ub;
        const bool better = cost < ub;
        if (better) {
            ub = cost;
            S->ub = ub;
        }
        S->steps += (unsigned long long)st;  // X-LAP steps stay in the scalar block
        S->best = fmax(S->best, lb);
        trace[S->t] = lb;
        S->t = S->t + 1;
        int proven = 0;
        if (ub < kInf) {
            const double tol = 1e-9 * fmax(1.0, fabs(ub));
            proven = integer_data ? (ceil(lb - tol) >= ub) : (ub - lb <= tol);
        }
        S->proven = proven;
        int stop = proven;
        if (min_gap > 0.0 && ub < kInf && ub != 0.0 && (ub - lb) / fabs(ub) < min_gap) stop = 1;
        S->stopped = stop;
        improved = better ? 1 : 0;
    }
    __syncthreads();
    const bool better = improved != 0;
    if (l < n) {
        xperm[l] = sig[l];
        if (better) bestperm[l] = sig[l];
    }
}

// ------------------------------------------------- Type 4 with annealing --
// Section 2.3's Type 4 rule under Section 5's annealing schedule, after the
// X-LAP of iteration it >= 1 (bound nu): a random fraction kappa^lb <=
// kappa_max of nu, split over one fraction per facility and per location in
// proportion to random weights, is offered to the x slacks (row i and
// column p grow uniformly, so every permutation's cost = LB + slacks still
// holds and the bound stays valid); the offer A is taken when
// u <= exp(-A / T), T = t0 * cool^floor(it / period), and LB drops by A.
// Draws: SplitMix64 outputs it*(2n+2) + 1 (size), + 2 (acceptance),
// + 3 ... + 2n+2 (weights, facilities then locations).
struct SaConsts {
    double t0, kmax, cool;
    unsigned long long seed;
    int period;
};

// c-th output (c >= 1) of SplitMix64 seeded with `seed` (Steele, Lea and
// Flood 2014: Weyl increment 0x9e3779b97f4a7c15 and its published
// finaliser), as a uniform double in [0, 1) from the top 53 bits.
__device__ __forceinline__ double sa_uniform(unsigned long long seed, unsigned long long c)
{
    unsigned long long z = seed + c * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// exp(x), x <= 0, in plain IEEE operations so that every platform computes
// the same bits: x = k ln2 + r (Cody-Waite with a 32-bit high part, k * high
// exact), degree-13 Taylor polynomial in Horner form, scaled by 2^k.
__device__ __forceinline__ double sa_exp(double x)
{
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double log2e = 1.44269504088896338700e+00;
    if (x < -745.0) return 0.0;
    const double k = floor(x * log2e + 0.5);
    const double r = (x - k * ln2_hi) - k * ln2_lo;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

// One wave; lane 0 draws and decides (2n <= 128 sequential terms, the
// summation order of the definition), all lanes then update pi_x.
__global__ __launch_bounds__(64) void k_type4(double *__restrict__ Px, DevScalars *__restrict__ S, int n,
                                              SaConsts K)
{
    if (S->stopped) return;
    __shared__ double w[128], a[128];
    __shared__ int take;
    const int l = threadIdx.x;
    if (l == 0) {
        take = 0;
        const int it = S->t - 1;  // the iteration whose X-LAP just ran
        const double nu = S->lb;
        if (it >= 1 && nu > 0.0) {
            const unsigned long long base = (unsigned long long)it * (unsigned long long)(2 * n + 2);
            const double us = sa_uniform(K.seed, base + 1);
            const double ua = sa_uniform(K.seed, base + 2);
            double W = 0.0;
            for (int k = 0; k < 2 * n; ++k) {
                w[k] = sa_uniform(K.seed, base + 3 + (unsigned long long)k);
                W = (k == 0) ? w[k] : W + w[k];
            }
            if (W > 0.0) {
                const double klb = K.kmax * us;
                double A = 0.0;
                for (int k = 0; k < 2 * n; ++k) {
                    a[k] = ((klb * w[k]) / W) * nu;
                    A = (k == 0) ? a[k] : A + a[k];
                }
                double T = K.t0;
                for (int c = 0; c < it / K.period; ++c) T = T * K.cool;
                if (ua <= sa_exp(-(A / T))) {
                    take = 1;
                    S->lb = nu - A;
                    S->sa_steps = S->sa_steps + 1;
                }
            }
        }
    }
    __syncthreads();
    if (take)
        for (int e = l; e < n * n; e += 64) Px[e] = (Px[e] + a[e / n]) + a[n + e % n];
}

// -------------------------------------------------------------- LAP batch --
template <int L, int C>
__global__ __launch_bounds__(256) void k_lap_batch(const double *__restrict__ cost, int count, int m,
                                                   double *__restrict__ uo, double *__restrict__ vo,
                                                   double *__restrict__ tho, int *__restrict__ rco)
{
    extern __shared__ double lds[];
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const int gbase = (threadIdx.x & 63) - l;
    const long long t0 = (long long)blockIdx.x * G;
    const int mm = m * m;
    const long long left = count - t0;
    const int nt = (int)(left < G ? left : G);
    const double *src = cost + t0 * mm;
    copy_to_lds(lds, src, nt * mm, threadIdx.x, blockDim.x);
    double *scr = lds + (size_t)G * mm + (size_t)g * 2 * m;
    __syncthreads();
    if (g < nt) {
        const long long t = t0 + g;
        double u[C], v[C], th;
        int pc[C], st = 0;
        lap_solve<L, C>(lds + (size_t)g * mm, m, l, gbase, scr, (int *)(scr + m), (int *)(scr + m) + m, u, v,
                        pc, th, st);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m) {
                uo[t * m + j] = u[c];
                vo[t * m + j] = v[c];
                rco[t * m + j] = pc[c];
            }
        }
        if (l == 0) tho[t] = th;
    }
}

}  // namespace qap
