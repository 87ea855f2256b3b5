// batch.hpp -- many independent dual ascents of uneven size n advanced in
// lockstep by one set of kernels per phase (the branch-and-bound nodes of
// Section 4 on one GPU), plus the child fold that warm-starts a node from its
// parent's reduced costs.
//
// A batch is a table of node descriptors.  Each per-phase kernel flattens the
// work of all nodes (tiles, Y-LAPs, orbit cubes, entries) into one grid; a
// block or lane group finds its node by binary search in a prefix table.
// Every node keeps its own iteration counter and stop flag in its DevScalars,
// so the same kernel sequence serves every iteration and is replayed from one
// HIP graph; a stopped node's jobs read its flag and leave, and the host drops
// stopped nodes from the tables as they accumulate.
//
// The arithmetic of every node is exactly that of the single-instance kernels
// in kernels.hpp (same expressions, same order), so a node's trajectory does
// not depend on what else is in its batch.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qap {

struct BNode {
    double *Z, *Yc, *Py, *Xc, *Px, *alpha, *beta, *trace;
    const double *F, *D, *B;
    int *xperm, *bestperm;
    DevScalars *S;
    unsigned long long *bins;
    const int *triples;
    long long T;
    int n, m, ntri, nb;
    int integer_data;
    int trace_cap;
    double offset, min_gap;
    double kz, okz, ky2, kx3, phi, oky, okx, phy, ophy;
};

// Node-level stop rules of a batch (branch-and-bound control, Section 4/5.4):
// besides the per-node min_gap and optimality certificate, a node stops when
// its bound fathoms against ub_cut, or when over `window` iterations its
// bound rose by less than min_improve * max(1, |UB|) (reason 2 = branch).
struct BatchCtl {
    double ub_cut;       // incumbent at batch start (+inf if none)
    double min_improve;  // 0 disables the window rule
    int window;
    int nnodes;
    int *nstopped;       // nodes that stopped during this batch (the host ends the batch when all have)
};

struct BatchPrefix {
    const long long *zl;  // tiles
    const long long *yl;  // Y-LAPs (n^2)
    const long long *sw;  // sweep blocks (triples * nb^3)
    const long long *sc;  // scale elements (T + n^2)
};

// A node's arrays are reached through pointers held in the node table, which
// the compiler cannot place in an address space: used as they are, their
// accesses are flat operations, and a flat access holds up every later LDS
// wait as well.  Held as global-space pointers they compile to global loads
// and stores.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> glob(T *p)
{
    return (gptr<T>)p;
}

__device__ __forceinline__ int find_node(const long long *pre, int nnodes, long long j)
{
    const gptr<const long long> p = glob(pre);
    int lo = 0, hi = nnodes - 1;  // largest b with pre[b] <= j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p[mid] <= j)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The node of job j >= the first job of node b0: step over the node ends in
// between.  Kernels whose lane groups hold different jobs find the node of
// the wavefront's first job once (find_node on a wave-uniform job runs on
// scalar loads, which the scalar cache serves) and each group steps from
// there, rather than each group searching with vector loads in turn.
__device__ __forceinline__ int find_node_from(const long long *pre, int nnodes, int b0, long long j)
{
    const gptr<const long long> p = glob(pre);
    int b = b0;
    while (b + 1 < nnodes && p[b + 1] <= j) ++b;
    return b;
}

// ----------------------------------------------------------------- sweep --
__global__ __launch_bounds__(256) void k_bsweep(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes)
{
    __shared__ double gs[6 * SB_CUBE];
    // XCD x (blocks are dealt to the 8 XCDs in turn) takes the x-th eighth of
    // the job numbers in order, so the cubes of one triple run on one XCD back
    // to back and the partial cache lines at run ends merge in its L2 (as in
    // k_sweep); the grid is the job count rounded up to a multiple of 8
    const long long G = glob(pf.sw)[nnodes], per = (G + 7) >> 3;
    const long long jb = (long long)(blockIdx.x & 7u) * per + (long long)(blockIdx.x >> 3);
    if (jb >= G) return;
    const int b = find_node(pf.sw, nnodes, jb);
    const BNode &N = nodes[b];
    if (glob(N.S)->stopped || glob(N.S)->t < 1) return;
    const int nb = N.nb, n = N.n;
    const int local = (int)(jb - glob(pf.sw)[b]);
    const int nb3 = nb * nb * nb;
    const int tri = local / nb3, sub = local % nb3;
    const int base[3] = {(sub / (nb * nb)) * SB, ((sub / nb) % nb) * SB, (sub % nb) * SB};
    const int packed = glob(N.triples)[tri];
    const int fi = packed & 0xff, fj = (packed >> 8) & 0xff, fk = (packed >> 16) & 0xff;
    const int m = N.m;
    const long long mm = (long long)m * m;
    const gptr<double> Z = glob(N.Z);
    const gptr<const double> Py = glob((const double *)N.Py), Px = glob((const double *)N.Px);
    const int F1[6] = {fi, fi, fj, fj, fk, fk};
    const int F2[6] = {fj, fk, fi, fk, fi, fj};
    const int F3[6] = {fk, fj, fk, fi, fj, fi};
    const int X1[6] = {0, 0, 1, 1, 2, 2};
    const int X2[6] = {1, 2, 0, 2, 0, 1};
    const int X3[6] = {2, 1, 2, 0, 1, 0};
    constexpr int PER = (SB * SB * SB) / 256;
    // pi_y of the block's tiles and pi_x of its (facility, location) pairs,
    // read once per block into registers and written to LDS after the z
    // loads have been issued (as k_sweep)
    __shared__ double pys[6 * SB * SB];
    __shared__ double pxs[3 * SB];
    constexpr int YREP = (6 * SB * SB + 255) / 256;
    double yv[YREP];
    double xv = 0.0;
#pragma unroll
    for (int rep = 0; rep < YREP; ++rep) {
        const int a = threadIdx.x + 256 * rep;
        yv[rep] = 0.0;
        if (a < 6 * SB * SB) {
            const int e = a / (SB * SB), a1 = (a / SB) % SB, a2 = a % SB;
            const int x1 = e >> 1, x2 = (0x102021 >> (4 * e)) & 0xf;  // X1[e], X2[e]
            const int f1 = x1 == 0 ? fi : (x1 == 1 ? fj : fk), f2 = x2 == 0 ? fi : (x2 == 1 ? fj : fk);
            const int l1 = (x1 == 0 ? base[0] : (x1 == 1 ? base[1] : base[2])) + a1;
            const int l2 = (x2 == 0 ? base[0] : (x2 == 1 ? base[1] : base[2])) + a2;
            yv[rep] = (l1 < n && l2 < n && l1 != l2) ? Py[tile_of(n, f1, l1, f2, l2)] : 0.0;
        }
    }
    if (threadIdx.x < 3 * SB) {
        const int x = threadIdx.x / SB, l = (x == 0 ? base[0] : (x == 1 ? base[1] : base[2])) + threadIdx.x % SB;
        const int f = x == 0 ? fi : (x == 1 ? fj : fk);
        xv = l < n ? Px[f * n + l] : 0.0;
    }
    long long za[6][PER];
    int li[6][PER];
    bool ok[6][PER];
    double pz[6][PER];
    // element addresses: the wave-uniform tile row and z row as a scalar
    // offset, l2' * m^2 + col per lane (as k_sweep)
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int a2 = (int)(threadIdx.x >> 3) & (SB - 1), a3 = (int)threadIdx.x & (SB - 1);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
#pragma unroll
        for (int w = 0; w < PER; ++w) {
            const int a1 = wid + (256 / (SB * SB)) * w;
            int loc[3];
            loc[X1[e]] = base[X1[e]] + a1;
            loc[X2[e]] = base[X2[e]] + a2;
            loc[X3[e]] = base[X3[e]] + a3;
            const int l1 = loc[X1[e]], l2 = loc[X2[e]], l3 = loc[X3[e]];
            const bool v = l1 < n && l2 < n && l3 < n && l1 != l2 && l1 != l3 && l2 != l3;
            const int f1 = F1[e], f2 = F2[e], f3 = F3[e];
            const int f2p = f2 - (f2 > f1);
            const int row = f3 - (f3 > f1) - (f3 > f2);
            const long long zrow = ((long long)(f1 * n + l1) * (n - 1) + f2p) * (n - 1) * mm + (long long)row * m;
            const int l2p = l2 - (l2 > l1);
            const int col = l3 - (l3 > l1) - (l3 > l2);
            ok[e][w] = v;
            za[e][w] = v ? zrow + (long long)(__umul24((unsigned)l2p, (unsigned)mm) + col) : 0;
            li[e][w] = cube_idx(loc[0] - base[0], loc[1] - base[1], loc[2] - base[2]);
            pz[e][w] = v ? Z[za[e][w]] : 0.0;
        }
    }
    // (every load above is issued before the first LDS write)
#pragma unroll
    for (int rep = 0; rep < YREP; ++rep) {
        const int a = threadIdx.x + 256 * rep;
        if (a < 6 * SB * SB) pys[a] = yv[rep];
    }
    if (threadIdx.x < 3 * SB) pxs[threadIdx.x] = xv;
#pragma unroll
    for (int e = 0; e < 6; ++e)
#pragma unroll
        for (int w = 0; w < PER; ++w)
            if (ok[e][w]) gs[e * SB_CUBE + li[e][w]] = pz[e][w];
    __syncthreads();
#pragma unroll
    for (int w = 0; w < PER; ++w) {
        const int u = threadIdx.x + 256 * w;
        const int rl = u % SB, ql = (u / SB) % SB, pl = u / (SB * SB);
        const int p = base[0] + pl, q = base[1] + ql, r = base[2] + rl;
        if (p < n && q < n && r < n && p != q && p != r && q != r) {
            const int c = cube_idx(pl, ql, rl);
            const int lc[3] = {pl, ql, rl};
            double g[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const double y = pys[(e * SB + lc[X1[e]]) * SB + lc[X2[e]]];
                const double x = pxs[X1[e] * SB + lc[X1[e]]];
                g[e] = (N.kz * gs[e * SB_CUBE + c] + N.ky2 * y) + N.kx3 * x;
            }
            gs[0 * SB_CUBE + c] = N.phi * ((((g[1] + g[2]) + g[3]) + g[4]) + g[5]);
            gs[1 * SB_CUBE + c] = N.phi * ((((g[0] + g[2]) + g[3]) + g[4]) + g[5]);
            gs[2 * SB_CUBE + c] = N.phi * ((((g[0] + g[1]) + g[3]) + g[4]) + g[5]);
            gs[3 * SB_CUBE + c] = N.phi * ((((g[0] + g[1]) + g[2]) + g[4]) + g[5]);
            gs[4 * SB_CUBE + c] = N.phi * ((((g[0] + g[1]) + g[2]) + g[3]) + g[5]);
            gs[5 * SB_CUBE + c] = N.phi * ((((g[0] + g[1]) + g[2]) + g[3]) + g[4]);
        }
    }
    __syncthreads();
    // every new value first (each slot's li is inside the cube, so the reads
    // for slots outside the instance stay in LDS and are discarded), then the
    // stores.  A new value needs pz, whose load was conditional: computed
    // inside its store's branch, it could only be waited for by waiting for
    // every outstanding memory operation, the earlier stores included, which
    // serialised the twelve stores.  The empty asm keeps each value out of
    // its store's branch.
    double nz[6][PER];
#pragma unroll
    for (int e = 0; e < 6; ++e)
#pragma unroll
        for (int w = 0; w < PER; ++w) {
            nz[e][w] = N.okz * pz[e][w] + gs[e * SB_CUBE + li[e][w]];
            asm volatile("" : "+v"(nz[e][w]));
        }
#pragma unroll
    for (int e = 0; e < 6; ++e)
#pragma unroll
        for (int w = 0; w < PER; ++w)
            if (ok[e][w]) Z[za[e][w]] = nz[e][w];
}

// The x/y scaling after the sweep has read pi_x, pi_y.
__global__ void k_bscale(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes)
{
    const long long total = glob(pf.sc)[nnodes];
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int b = find_node(pf.sc, nnodes, e);
        const BNode &N = nodes[b];
        if (glob(N.S)->stopped || glob(N.S)->t < 1) continue;
        const long long a = e - glob(pf.sc)[b];
        if (a < N.T)
            glob(N.Yc)[a] = N.oky * glob(N.Py)[a];
        else
            glob(N.Xc)[a - N.T] = N.okx * glob(N.Px)[a - N.T];
    }
}

// ----------------------------------------------------------------- Z-LAP --
// One group of L lanes per tile; LDS per group sized for the batch's largest m.
template <int L>
__global__ __launch_bounds__(256) void k_bzlap(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes,
                                               int mmax)
{
    extern __shared__ double lds[];
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const int gbase = (threadIdx.x & 63) - l;
    const long long jg = (long long)blockIdx.x * G + g;
    const int per = mmax * mmax + 2 * mmax;
    double *M = lds + (size_t)g * per;
    const long long total = glob(pf.zl)[nnodes];
    // the wavefront finds the node of its first group's tile, each group
    // steps from there to its own
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long jw = (long long)blockIdx.x * G + (long long)wv * (64 / L);
    const int bw = find_node(pf.zl, nnodes, jw < total ? jw : total - 1);
    bool live = jg < total;
    int b = 0;
    if (live) {
        b = find_node_from(pf.zl, nnodes, bw, jg);
        live = !glob(nodes[b].S)->stopped;
    }
    if (!live) return;  // whole groups leave together; no block barrier below
    const BNode &N = nodes[b];
    const int m = N.m, mm = m * m;
    const long long t = jg - glob(pf.zl)[b];
    const gptr<double> src = glob(N.Z) + t * mm, Yc = glob(N.Yc);
    copy_to_lds(M, (const double *)src, mm, l, L);
    const double yc0 = Yc[t];  // read now, added to after the solve
    double *lu = M + mm;
    int *lp = (int *)(lu + m);
    int *lw = lp + m;
    __builtin_amdgcn_wave_barrier();
    double u[1], v[1], th;
    int pc[1], st = 0;
    lap_solve<L, 1>(M, m, l, gbase, lu, lp, lw, u, v, pc, th, st);
    __builtin_amdgcn_wave_barrier();
    double *vs = lu + m;
    if (l < m) vs[l] = v[0];
    __builtin_amdgcn_wave_barrier();
    // slacks back in place, row by row (no division per element)
    for (int col = l; col < m; col += L) {
        const double vc = vs[col];
#pragma unroll 2
        for (int r = 0; r < m; ++r) src[r * m + col] = (M[r * m + col] - lu[r]) - vc;
    }
    if (l == 0) {
        Yc[t] = yc0 + th;
        atomicAdd((unsigned long long *)(glob(N.bins) + (jg & (kStepBins - 1))), (unsigned long long)st);
    }
}

// Batched Z-LAPs with the scalar-controlled solver (m <= 32): one wavefront
// per tile, its node found by binary search as in k_bzlap; the work per tile
// is k_zlap_s<1>'s, in the same order.
__global__ __launch_bounds__(64) void k_bzlap_s(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes)
{
    extern __shared__ double lds[];
    const long long jg = blockIdx.x;
    if (jg >= glob(pf.zl)[nnodes]) return;
    const int b = find_node(pf.zl, nnodes, jg);
    const BNode &N = nodes[b];
    if (glob(N.S)->stopped) return;  // the whole block (one wave) leaves together
    const int lane = threadIdx.x;
    const int m = N.m, mm = m * m;
    const long long t = jg - glob(pf.zl)[b];
    const gptr<double> src = glob(N.Z) + t * mm, Yc = glob(N.Yc);
    copy_to_lds(lds, (const double *)src, mm, lane, 64);
    const double yc0 = Yc[t];  // read now, added to after the solve
    __syncthreads();
    double u, v, th;
    int p, st;
    if (m <= 16)
        lap_solve_scalar1<16>(lds, 0, mm, m, u, v, p, th, st);
    else
        lap_solve_scalar1<32>(lds, 0, mm, m, u, v, p, th, st);
    __builtin_amdgcn_wave_barrier();
    double *scr = lds + mm;  // row potentials; v over the matching/links area
    if (lane < m) scr[m + lane] = v;
    __syncthreads();
    // slacks back in place; the two half-waves take alternate rows
    const int sub = lane >> 5, col = lane & 31;
    if (col < m) {
        const double vc = scr[m + col];
        for (int r = sub; r < m; r += 2) src[r * m + col] = (lds[r * m + col] - scr[r]) - vc;
    }
    if (lane == 0) {
        Yc[t] = yc0 + th;
        atomicAdd((unsigned long long *)(glob(N.bins) + (jg & (kStepBins - 1))), (unsigned long long)st);
    }
}

// Two tiles per wavefront (m <= 32): wave w takes tiles 2w and 2w+1, which
// belong to one node (every node has an even number of tiles, n^2 (n-1)^2,
// so every node's first tile is even); the work per tile is k_zlap_s<2>'s.
__global__ __launch_bounds__(64) void k_bzlap_s2(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes)
{
    extern __shared__ double lds[];
    const long long j0 = 2 * (long long)blockIdx.x;
    if (j0 >= glob(pf.zl)[nnodes]) return;
    const int b = find_node(pf.zl, nnodes, j0);
    const BNode &N = nodes[b];
    if (glob(N.S)->stopped) return;
    const int lane = (int)(threadIdx.x & 63);
    const int h = lane >> 5, l = lane & 31;
    const int m = N.m, mm = m * m;
    const long long t0 = j0 - glob(pf.zl)[b];
    const gptr<double> src = glob(N.Z) + t0 * mm, Yc = glob(N.Yc);
    copy_to_lds(lds, (const double *)src, 2 * mm, lane, 64);
    const double yc0 = Yc[t0 + h];  // read now, added to after the solve
    double *scr = lds + 2 * mm;
    const int toff[2] = {0, mm}, soff[2] = {2 * mm, 2 * mm + 2 * m};
    __syncthreads();
    double u, v, th;
    int p, st;
    if (m <= 16)
        lap_solve_scalar2<16>(lds, toff, soff, m, 2, u, v, p, th, st);
    else
        lap_solve_scalar2<32>(lds, toff, soff, m, 2, u, v, p, th, st);
    __builtin_amdgcn_wave_barrier();
    if (l < m) scr[h * 2 * m + m + l] = v;
    __syncthreads();
    if (l < m) {
        const double *us = scr + h * 2 * m;
        const double vc = us[m + l];
        const double *tl = lds + h * mm;
        const gptr<double> dst = src + h * mm;
        for (int r = 0; r < m; ++r) dst[r * m + l] = (tl[r * m + l] - us[r]) - vc;
    }
    if (l == 0) Yc[t0 + h] = yc0 + th;
    const int stt = __builtin_amdgcn_readlane(st, 0) + __builtin_amdgcn_readlane(st, 32);
    if (lane == 0) atomicAdd((unsigned long long *)(glob(N.bins) + (j0 & (kStepBins - 1))), (unsigned long long)stt);
}

// ----------------------------------------------------------------- Y-LAP --
template <int L>
__global__ __launch_bounds__(256) void k_bylap(const BNode *__restrict__ nodes, BatchPrefix pf, int nnodes,
                                               int mmax)
{
    extern __shared__ double lds[];
    const int G = blockDim.x / L;
    const int g = threadIdx.x / L, l = threadIdx.x % L;
    const int gbase = (threadIdx.x & 63) - l;
    const long long jg = (long long)blockIdx.x * G + g;
    const int per = mmax * mmax + 2 * mmax;
    double *M = lds + (size_t)g * per;
    const long long total = glob(pf.yl)[nnodes];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long jw = (long long)blockIdx.x * G + (long long)wv * (64 / L);
    const int bw = find_node(pf.yl, nnodes, jw < total ? jw : total - 1);
    bool live = jg < total;
    int b = 0;
    if (live) {
        b = find_node_from(pf.yl, nnodes, bw, jg);
        live = !glob(nodes[b].S)->stopped;
    }
    if (!live) return;
    const BNode &N = nodes[b];
    const int n = N.n, m = n - 1, mm = m * m;
    const int ip = (int)(jg - glob(pf.yl)[b]);
    const int i = ip / n, p = ip % n;
    const bool equalize = glob(N.S)->t >= 1;
    const long long base = (long long)ip * mm;
    const gptr<const double> Yc = glob((const double *)N.Yc);
    const gptr<double> Xc = glob(N.Xc), Py = glob(N.Py);
    const double xc0 = Xc[ip];  // read now, added to after the solve
    for (int e0 = 0; e0 < mm; e0 += 8 * L) {
        double av[8], bv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + l + L * k;
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
            const int e = e0 + l + L * k;
            if (e < mm) M[e] = equalize ? N.ophy * av[k] + N.phy * bv[k] : av[k];
        }
    }
    double *lu = M + mm;
    int *lp = (int *)(lu + m);
    int *lw = lp + m;
    __builtin_amdgcn_wave_barrier();
    double u[1], v[1], th;
    int pc[1], st = 0;
    lap_solve<L, 1>(M, m, l, gbase, lu, lp, lw, u, v, pc, th, st);
    __builtin_amdgcn_wave_barrier();
    double *vs = lu + m;
    if (l < m) vs[l] = v[0];
    __builtin_amdgcn_wave_barrier();
    for (int col = l; col < m; col += L) {
        const double vc = vs[col];
#pragma unroll 2
        for (int r = 0; r < m; ++r) Py[base + r * m + col] = (M[r * m + col] - lu[r]) - vc;
    }
    if (l == 0) {
        Xc[ip] = xc0 + th;
        atomicAdd((unsigned long long *)(glob(N.bins) + (jg & (kStepBins - 1))), (unsigned long long)st);
    }
}

// Scalar blocks of several handles gathered into one array, for one copy to
// the host.
__global__ void k_bgather_scalars(DevScalars *const *__restrict__ src, int count, DevScalars *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = *src[i];
}

// Each node's stop flag, for the host to drop stopped nodes from the tables.
__global__ void k_bstopped(const BNode *__restrict__ nodes, int nnodes, int *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnodes) out[i] = glob(nodes[i].S)->stopped;
}

// ----------------------------------------------------------------- X-LAP --
// One wavefront per node: the single-instance X-LAP step (bound, incumbent
// with the node's constant offset, certificate, min_gap) plus the batch's
// fathoming and window rules.  S->reason: 1 = optimality certificate or
// fathomed, 2 = window rule, 3 = min_gap.
__global__ __launch_bounds__(64) void k_bxlap(const BNode *__restrict__ nodes, BatchCtl ctl)
{
    const BNode &N = nodes[blockIdx.x];
    const gptr<DevScalars> S = glob(N.S);
    if (S->stopped) return;
    // the cost matrix, then the solver's scratch (as k_xlap)
    __shared__ double M[64 * 64 + 64 + 32];
    __shared__ double vs[64];
    __shared__ int sig[64];
    __shared__ int improved;
    const int l = threadIdx.x;
    const int n = N.n, nn = n * n;
    copy_to_lds(M, (const double *)glob((const double *)N.Xc), nn, l, 64);
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
        glob(N.alpha)[l] = u;
        glob(N.beta)[l] = v;
        sig[pc] = l;
    }
    __syncthreads();
    const double *lu = M + nn;  // the row potentials
    for (int e = l; e < nn; e += 64) glob(N.Px)[e] = (M[e] - lu[e / n]) - vs[e % n];
    double cd = 0.0;
    long long ci = 0;
    if (l < n) {
        const int si = sig[l];
        if (N.integer_data) {
            ci = (long long)glob(N.B)[l * n + si];
            for (int jj = 0; jj < n; ++jj) ci += (long long)glob(N.F)[l * n + jj] * (long long)glob(N.D)[si * n + sig[jj]];
        } else {
            cd = glob(N.B)[l * n + si];
            for (int jj = 0; jj < n; ++jj) cd = cd + glob(N.F)[l * n + jj] * glob(N.D)[si * n + sig[jj]];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ci += __shfl_xor(ci, off, 64);
        cd += __shfl_xor(cd, off, 64);
    }
    if (l == 0) {
        const double cost = (N.integer_data ? (double)ci : cd) + N.offset;
        const double lb = S->lb + th;
        S->lb = lb;
        double ub = S->ub;
        const bool better = cost < ub;
        if (better) {
            ub = cost;
            S->ub = ub;
        }
        S->steps += (unsigned long long)st;
        S->best = fmax(S->best, lb);
        const int t = S->t;
        if (t < N.trace_cap) glob(N.trace)[t] = lb;
        S->t = t + 1;
        int proven = 0;
        if (ub < kInf) {
            const double tol = 1e-9 * fmax(1.0, fabs(ub));
            proven = N.integer_data ? (ceil(lb - tol) >= ub) : (ub - lb <= tol);
        }
        S->proven = proven;
        int stop = proven, reason = proven ? 1 : 0;
        if (!stop && N.min_gap > 0.0 && ub < kInf && ub != 0.0 && (ub - lb) / fabs(ub) < N.min_gap) {
            stop = 1;
            reason = 3;
        }
        const double cut = ub < ctl.ub_cut ? ub : ctl.ub_cut;
        if (!stop && cut < kInf) {
            const double tol = 1e-9 * fmax(1.0, fabs(cut));
            const bool fath = N.integer_data ? (ceil(lb - tol) >= cut) : (lb >= cut - tol);
            if (fath) {
                stop = 1;
                reason = 1;
            }
        }
        if (!stop && ctl.min_improve > 0.0 && t + 1 > ctl.window && t + 1 - ctl.window - 1 >= 0 &&
            t + 1 - ctl.window - 1 < N.trace_cap) {
            const double ref = (cut < kInf) ? fabs(cut) : fabs(lb);
            if (lb - glob(N.trace)[t - ctl.window] < ctl.min_improve * fmax(1.0, ref)) {
                stop = 1;
                reason = 2;
            }
        }
        S->stopped = stop;
        S->reason = reason;
        if (stop) atomicAdd(ctl.nstopped, 1);
        improved = better ? 1 : 0;
    }
    __syncthreads();
    if (l < n) {
        glob(N.xperm)[l] = sig[l];
        if (improved) glob(N.bestperm)[l] = sig[l];
    }
}

// ----------------------------------------------------------------- fold ---
// Child of a parent in F-form (after >= 1 iteration: Px = pi_x, Py = pi_y,
// Z = pi_z) for fixing local facility l to local location s: entries holding
// (l,s) drop one level, the rest is restricted (see the oracle's fold).
__global__ void k_fold_xy(const double *__restrict__ pPx, const double *__restrict__ pPy,
                          const double *__restrict__ pZ, int n, int l, int s, double *__restrict__ cXc,
                          double *__restrict__ cYc)
{
    const int n1 = n - 1, m = n - 2;
    const long long mm = (long long)m * m;
    const long long T1 = (long long)n1 * n1 * (n1 - 1) * (n1 - 1);
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < T1 + (long long)n1 * n1;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < T1) {
            const int m1 = n1 - 1;
            const int qp = (int)(e % m1), jp = (int)((e / m1) % m1);
            const int ipc = (int)(e / ((long long)m1 * m1));
            const int a1 = ipc / n1, b1 = ipc % n1;
            const int a2 = jp + (jp >= a1), b2 = qp + (qp >= b1);
            const int i = a1 + (a1 >= l), p = b1 + (b1 >= s), j = a2 + (a2 >= l), q = b2 + (b2 >= s);
            const long long t1 = tile_of(n, l, s, i, p);   // z(l,i,j,s,p,q): row j, col q
            const long long t2 = tile_of(n, i, p, l, s);   // z(i,l,j,p,s,q): row j, col q
            const long long t3 = tile_of(n, i, p, j, q);   // z(i,j,l,p,q,s): row l, col s
            const double z1 = pZ[t1 * mm + (long long)(j - (j > l) - (j > i)) * m + (q - (q > s) - (q > p))];
            const double z2 = pZ[t2 * mm + (long long)(j - (j > i) - (j > l)) * m + (q - (q > p) - (q > s))];
            const double z3 = pZ[t3 * mm + (long long)(l - (l > i) - (l > j)) * m + (s - (s > p) - (s > q))];
            cYc[e] = ((pPy[t3] + z1) + z2) + z3;
        } else {
            const long long x = e - T1;
            const int a1 = (int)(x / n1), b1 = (int)(x % n1);
            const int i = a1 + (a1 >= l), p = b1 + (b1 >= s);
            cXc[x] = (pPx[i * n + p] + pPy[tile_of(n, l, s, i, p)]) + pPy[tile_of(n, i, p, l, s)];
        }
    }
}

__global__ void k_fold_z(const double *__restrict__ pZ, int n, int l, int s, double *__restrict__ cZ)
{
    const int n1 = n - 1, m = n - 2, m1 = n1 - 2;
    const long long mm = (long long)m * m, mm1 = (long long)m1 * m1;
    const long long V1 = (long long)n1 * n1 * (n1 - 1) * (n1 - 1) * mm1;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < V1;
         e += (long long)gridDim.x * blockDim.x) {
        const long long tc = e / mm1;
        const int w = (int)(e % mm1);
        const int rr = w / m1, cc = w % m1;
        const int q1 = n1 - 1;
        const int qp = (int)(tc % q1), jp = (int)((tc / q1) % q1);
        const int ipc = (int)(tc / ((long long)q1 * q1));
        const int a1 = ipc / n1, b1 = ipc % n1;
        const int a2 = jp + (jp >= a1), b2 = qp + (qp >= b1);
        // child row rr -> child facility a3 (skipping a1, a2), column cc -> b3
        const int flo = a1 < a2 ? a1 : a2, fhi = a1 < a2 ? a2 : a1;
        int a3 = rr;
        a3 += (a3 >= flo);
        a3 += (a3 >= fhi);
        const int llo = b1 < b2 ? b1 : b2, lhi = b1 < b2 ? b2 : b1;
        int b3 = cc;
        b3 += (b3 >= llo);
        b3 += (b3 >= lhi);
        const int i = a1 + (a1 >= l), j = a2 + (a2 >= l), k = a3 + (a3 >= l);
        const int p = b1 + (b1 >= s), q = b2 + (b2 >= s), r = b3 + (b3 >= s);
        const long long tp = tile_of(n, i, p, j, q);
        cZ[e] = pZ[tp * mm + (long long)(k - (k > i) - (k > j)) * m + (r - (r > p) - (r > q))];
    }
}

}  // namespace qap
