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
//   k_ylap        y-pair rule (Eq. da:yrule1) fused into the load, then the
//                 Y-LAPs (Delta_ip, gamma, delta)
//   k_xlap        the X-LAP, bound, incumbent, feasibility check, stop flag
//
// Device layout (see include/qap_rlt2.h): tiles t(i,p,j,q) =
// ((i*n+p)*(n-1)+j')*(n-1)+q'; z entries tile-major with compressed row k''
// and column r''.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lap_wave.hpp"

namespace qap {

struct DevScalars {
    double lb;
    double ub;
    int t;             // iterations completed
    int proven;
    int integer_data;
    int stopped;       // set once the bound proves optimality or gap < min_gap
    unsigned long long steps;
};

struct SweepConsts {
    double kz, okz, ky2, kx3, phi;
};

// Tile index of the ordered pair ((f1,l1),(f2,l2)), f1 != f2, l1 != l2.
__device__ __forceinline__ long long tile_of(int n, int f1, int l1, int f2, int l2)
{
    const int f2p = f2 - (f2 > f1);
    const int l2p = l2 - (l2 > l1);
    return ((long long)(f1 * n + l1) * (n - 1) + f2p) * (n - 1) + l2p;
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
// tile and its x parent P1.  With pi_z(e) = (R_z(e) - u_row) - v_col from the
// last Z-LAP duals:
//   g_e   = (kz*pi_z(e) + ky2*pi_y(tile(e))) + kx3*pi_x(P1(e))
//   new_e = okz*pi_z(e) + phi*(left fold of g_f over f != e, canonical order)
//
// One block per (facility triple, location p of the first facility); the
// thread loop covers the (n-1)(n-2) orbits (q, r).  Blocks are numbered so
// that the n blocks of one triple land on the same XCD back to back: lanes
// walk r, so members (A,B,C) and (B,A,C) read whole tile rows, members
// (A,C,B)/(C,A,B) reuse their rows over the q loop inside the block, and
// members (B,C,A)/(C,B,A) share their cache lines with the neighbouring p
// blocks of the same triple in that XCD's L2.
__global__ __launch_bounds__(256) void k_sweep(double *__restrict__ Z, const double *__restrict__ U,
                                               const double *__restrict__ V,
                                               const double *__restrict__ Py,
                                               const double *__restrict__ Px,
                                               const int *__restrict__ triples, int ntriples, int n,
                                               SweepConsts K, const DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    const unsigned b = blockIdx.x;
    const unsigned xcd = b & 7u, s = b >> 3;
    const int p = (int)(s % (unsigned)n);
    const int tri = (int)((s / (unsigned)n) * 8u + xcd);
    if (tri >= ntriples) return;
    const int packed = triples[tri];
    const int i = packed & 0xff, j = (packed >> 8) & 0xff, k = (packed >> 16) & 0xff;
    const int m = n - 2;
    const long long mm = (long long)m * m;
    const int norb = (n - 1) * m;
    for (int o = threadIdx.x; o < norb; o += blockDim.x) {
        const int qp = o / m, rr = o % m;
        const int q = qp + (qp >= p);
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        int r = rr;
        r += (r >= lo);
        r += (r >= hi);
        const int fa[3] = {i, j, k};
        const int la[3] = {p, q, r};
        // canonical member order as index triples into (A,B,C)
        const int o1[6] = {0, 0, 1, 1, 2, 2};
        const int o2[6] = {1, 2, 0, 2, 0, 1};
        const int o3[6] = {2, 1, 2, 0, 1, 0};
        long long za[6];
        double pz[6], g[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int f1 = fa[o1[e]], l1 = la[o1[e]];
            const int f2 = fa[o2[e]], l2 = la[o2[e]];
            const int f3 = fa[o3[e]], l3 = la[o3[e]];
            const long long t = tile_of(n, f1, l1, f2, l2);
            const int row = f3 - (f3 > f1) - (f3 > f2);
            const int col = l3 - (l3 > l1) - (l3 > l2);
            za[e] = t * mm + (long long)row * m + col;
            pz[e] = (Z[za[e]] - U[t * m + row]) - V[t * m + col];
            g[e] = (K.kz * pz[e] + K.ky2 * Py[t]) + K.kx3 * Px[f1 * n + l1];
        }
        const double n0 = ((((g[1] + g[2]) + g[3]) + g[4]) + g[5]);
        const double n1 = ((((g[0] + g[2]) + g[3]) + g[4]) + g[5]);
        const double n2 = ((((g[0] + g[1]) + g[3]) + g[4]) + g[5]);
        const double n3 = ((((g[0] + g[1]) + g[2]) + g[4]) + g[5]);
        const double n4 = ((((g[0] + g[1]) + g[2]) + g[3]) + g[5]);
        const double n5 = ((((g[0] + g[1]) + g[2]) + g[3]) + g[4]);
        Z[za[0]] = K.okz * pz[0] + K.phi * n0;
        Z[za[1]] = K.okz * pz[1] + K.phi * n1;
        Z[za[2]] = K.okz * pz[2] + K.phi * n2;
        Z[za[3]] = K.okz * pz[3] + K.phi * n3;
        Z[za[4]] = K.okz * pz[4] + K.phi * n4;
        Z[za[5]] = K.okz * pz[5] + K.phi * n5;
    }
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
// Groups of L lanes, G = blockDim/L groups per block; the block copies its G
// consecutive tiles (contiguous in HBM) into LDS with one coalesced loop.
// Writes xi (row duals) to U, psi (column duals) to V, adds Theta to R_y.
template <int L, int C>
__global__ __launch_bounds__(256) void k_zlap(const double *__restrict__ Z, double *__restrict__ U,
                                              double *__restrict__ V, double *__restrict__ Yc, int m,
                                              long long T, DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    extern __shared__ double lds[];
    __shared__ unsigned long long bsteps;
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const long long t0 = (long long)blockIdx.x * G;
    const int mm = m * m;
    const long long left = T - t0;
    const int nt = (int)(left < G ? left : G);
    const double *src = Z + t0 * mm;
    for (int e = threadIdx.x; e < nt * mm; e += blockDim.x) lds[e] = src[e];
    if (threadIdx.x == 0) bsteps = 0ull;
    __syncthreads();
    const long long t = t0 + g;
    int st = 0;
    if (g < nt) {
        double u[C], v[C], th;
        int pc[C];
        lap_solve<L, C>(lds + g * mm, m, m, l, u, v, pc, th, st);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m) {
                U[t * m + j] = u[c];
                V[t * m + j] = v[c];
            }
        }
        if (l == 0) {
            Yc[t] = Yc[t] + th;
            atomicAdd(&bsteps, (unsigned long long)st);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&S->steps, bsteps);
}

// ----------------------------------------------------------------- Y-LAP --
// One group per (i,p); its (n-1)x(n-1) block of R_y is contiguous.  For
// t >= 1 every entry is first replaced by ophy*R_y[ijpq] + phy*R_y[jiqp]
// (the y-pair rule applied by both members of the pair).  Writes pi_y to Py
// and adds Delta_ip to R_x.
template <int L, int C>
__global__ __launch_bounds__(256) void k_ylap(const double *__restrict__ Yc, double *__restrict__ Py,
                                              double *__restrict__ Xc, int n, int equalize,
                                              double ophy, double phy, DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    extern __shared__ double lds[];
    __shared__ unsigned long long bsteps;
    const int m = n - 1, mm = m * m;
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const int ip = blockIdx.x * G + g;
    // per group: matrix (mm) + u (m) + v (m)
    double *M = lds + (size_t)g * (mm + 2 * m);
    double *us = M + mm;
    double *vs = us + m;
    if (threadIdx.x == 0) bsteps = 0ull;
    const bool active = ip < n * n;
    if (active) {
        const int i = ip / n, p = ip % n;
        const long long base = (long long)ip * mm;
        for (int e = l; e < mm; e += L) {
            double a = Yc[base + e];
            if (equalize) {
                const int jp = e / m, qp = e % m;
                const int j = jp + (jp >= i), q = qp + (qp >= p);
                const long long tb = ((long long)(j * n + q) * m + (i - (i > j))) * m + (p - (p > q));
                a = ophy * a + phy * Yc[tb];
            }
            M[e] = a;
        }
    }
    __syncthreads();
    if (active) {
        double u[C], v[C], th;
        int pc[C], st = 0;
        lap_solve<L, C>(M, m, m, l, u, v, pc, th, st);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = l + L * c;
            if (j < m) {
                us[j] = u[c];
                vs[j] = v[c];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const long long base = (long long)ip * mm;
        for (int e = l; e < mm; e += L) Py[base + e] = (M[e] - us[e / m]) - vs[e % m];
        if (l == 0) {
            Xc[ip] = Xc[ip] + th;
            atomicAdd(&bsteps, (unsigned long long)st);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&S->steps, bsteps);
}

// ----------------------------------------------------------------- X-LAP --
// One wave.  LB += theta_x; pi_x -> Px; alpha/beta; the assignment is a QAP
// solution whose exact cost (int64 for integer data) updates the incumbent;
// feasibility check and gap test set the stop flag.
__global__ __launch_bounds__(64) void k_xlap(const double *__restrict__ Xc, double *__restrict__ Px,
                                             double *__restrict__ alpha, double *__restrict__ beta,
                                             const double *__restrict__ F, const double *__restrict__ D,
                                             const double *__restrict__ B, int *__restrict__ xperm,
                                             int *__restrict__ bestperm, double *__restrict__ trace,
                                             int n, double min_gap, DevScalars *__restrict__ S)
{
    if (S->stopped) return;
    __shared__ double M[64 * 64];
    __shared__ double us[64], vs[64];
    __shared__ int sig[64];
    __shared__ int improved;
    const int l = threadIdx.x;
    const int nn = n * n;
    for (int e = l; e < nn; e += 64) M[e] = Xc[e];
    __syncthreads();
    double u[1], v[1], th;
    int pc[1], st = 0;
    lap_solve<64, 1>(M, n, n, l, u, v, pc, th, st);
    if (l < n) {
        us[l] = u[0];
        vs[l] = v[0];
        alpha[l] = u[0];
        beta[l] = v[0];
        sig[pc[0]] = l;
    }
    __syncthreads();
    for (int e = l; e < nn; e += 64) Px[e] = (M[e] - us[e / n]) - vs[e % n];
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
        const double cost = integer_data ? (double)ci : cd;
        const double lb = S->lb + th;
        S->lb = lb;
        double ub = S->ub;
        const bool better = cost < ub;
        if (better) {
            ub = cost;
            S->ub = ub;
        }
        S->steps += (unsigned long long)st;
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

// -------------------------------------------------------------- LAP batch --
template <int L, int C>
__global__ __launch_bounds__(256) void k_lap_batch(const double *__restrict__ cost, int count, int m,
                                                   double *__restrict__ uo, double *__restrict__ vo,
                                                   double *__restrict__ tho, int *__restrict__ rco)
{
    extern __shared__ double lds[];
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const long long t0 = (long long)blockIdx.x * G;
    const int mm = m * m;
    const long long left = count - t0;
    const int nt = (int)(left < G ? left : G);
    const double *src = cost + t0 * mm;
    for (int e = threadIdx.x; e < nt * mm; e += blockDim.x) lds[e] = src[e];
    __syncthreads();
    if (g < nt) {
        const long long t = t0 + g;
        double u[C], v[C], th;
        int pc[C], st = 0;
        lap_solve<L, C>(lds + g * mm, m, m, l, u, v, pc, th, st);
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
