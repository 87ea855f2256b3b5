// learn.hpp -- device kernels of the learned warm start.
//
// The z variables come in orbits of six tied by the symmetry constraints
// (Eq. rlt2:con3): the orderings of one set {A=(i,p), B=(j,q), C=(k,r)},
// i<j<k, p,q,r distinct.  Any multipliers v that sum to zero over every
// orbit are valid in the Lagrangian dual (Section 3.1), so a start from z
// costs -v gives a valid bound whatever v is.  A three-layer perceptron maps
// 32 per-orbit features to six outputs; their zero-sum projection, scaled,
// is v.
//
// Orbit ids: o = tri * n(n-1)(n-2) + (p*(n-1) + q')*(n-2) + r'', tri the
// index of (i,j,k) among the facility triples in lexicographic order, q' and
// r'' compressed past the smaller locations.  Members in the canonical order
// (A,B,C),(A,C,B),(B,A,C),(B,C,A),(C,A,B),(C,B,A), as in the sweep.
//
// Kernels:
//   k_orbit_features   features of listed orbits (training inputs)
//   k_orbit_targets    tracked multipliers of listed orbits / scale
//   k_orbit_mlp        features + perceptron over all orbits, weights held in
//                      LDS as bf16 MFMA fragments (32x32x16), one persistent
//                      block per CU; hidden activations stay in registers
//   k_warm_z           outputs -> zero-sum multipliers -> z costs -v, written
//                      through the sweep's LDS cube transpose
//   k_gemm             bf16 MFMA GEMM with strided operands and the epilogues
//                      of the training step
//   k_out_err, k_rowsum, k_adam, k_mlp_pack   the rest of the training step
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qap {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kFeat = 32;   // perceptron inputs (28 used)
constexpr int kWidth = 256; // hidden width
constexpr int kOut = 6;     // outputs, one per orbit member

// Parameter block (float32 masters, gradients and Adam moments share it).
constexpr int kOffW1 = 0;                          // W1 [256][32]
constexpr int kOffB1 = kOffW1 + kWidth * kFeat;    // b1 [256]
constexpr int kOffW2 = kOffB1 + kWidth;            // W2 [256][256]
constexpr int kOffB2 = kOffW2 + kWidth * kWidth;   // b2 [256]
constexpr int kOffW3 = kOffB2 + kWidth;            // W3 [6][256]
constexpr int kOffB3 = kOffW3 + kOut * kWidth;     // b3 [6]
constexpr int kParams = kOffB3 + kOut;             // 75782

// bf16 copies: row-major GEMM copies (W1, W2, W3 back to back) and the MFMA
// fragment copies of the fused kernel.
constexpr int kRowW1 = 0, kRowW2 = kWidth * kFeat, kRowW3 = kRowW2 + kWidth * kWidth;
constexpr int kRowTotal = kRowW3 + kOut * kWidth;
// fragments, in units of 8 bf16 (16 bytes, one lane's operand)
constexpr int kFragW1 = 0;                       // [mb 8][chunk 2][lane 64]
constexpr int kFragW2 = kFragW1 + 8 * 2 * 64;    // [mb 8][chunk 16][lane 64]
constexpr int kFragW3 = kFragW2 + 8 * 16 * 64;   // [chunk 16][half 2][row 6]
constexpr int kFragTotal = kFragW3 + 16 * 2 * 6; // 9408 x 16 B = 150528 B

// Input feature of hidden slot i in the K-chunk c of layers 2 and 3.  The
// 32x32x16 MFMA leaves lane (col, half h) of M-block mb holding rows
// 32 mb + 8 (j/4) + 4 h + (j%4), j = 0..15; taking j = 8a + i as slot i of
// chunk c = 2 mb + a lets the next layer use those registers as its B
// operand unchanged, with the weights' K order permuted to match.
__host__ __device__ inline int chunk_feature(int c, int h, int i)
{
    return 32 * (c >> 1) + 16 * (c & 1) + 8 * (i >> 2) + 4 * h + (i & 3);
}

struct FeatTables {
    const float *Fn, *Dn, *Xn, *fa, *dl;  // n*n, n*n, n*n, n, n
    float fbar, dbar, inv_m;
    int n;
};

__device__ __forceinline__ void decode_orbit(long long o, int n, const int *__restrict__ triples, int &i,
                                             int &j, int &k, int &p, int &q, int &r)
{
    const int nm1 = n - 1, nm2 = n - 2;
    const long long L3 = (long long)n * nm1 * nm2;
    const long long tri = o / L3;
    const int rest = (int)(o - tri * L3);
    const int packed = triples[tri];
    i = packed & 0xff;
    j = (packed >> 8) & 0xff;
    k = (packed >> 16) & 0xff;
    p = rest / (nm1 * nm2);
    const int qq = (rest / nm2) % nm1;
    const int rr = rest % nm2;
    q = qq + (qq >= p);
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    r = rr + (rr >= lo);
    r += (r >= hi);
}

// The 32 inputs of orbit (i,j,k,p,q,r); see the oracle's feature list.
__device__ __forceinline__ void orbit_features(const FeatTables &T, int i, int j, int k, int p, int q, int r,
                                               float f[kFeat])
{
    const int n = T.n;
    const float fij = T.Fn[i * n + j], fji = T.Fn[j * n + i], fik = T.Fn[i * n + k], fki = T.Fn[k * n + i];
    const float fjk = T.Fn[j * n + k], fkj = T.Fn[k * n + j];
    const float dpq = T.Dn[p * n + q], dqp = T.Dn[q * n + p], dpr = T.Dn[p * n + r], drp = T.Dn[r * n + p];
    const float dqr = T.Dn[q * n + r], drq = T.Dn[r * n + q];
    f[0] = fij * dpq;
    f[1] = fji * dqp;
    f[2] = fik * dpr;
    f[3] = fki * drp;
    f[4] = fjk * dqr;
    f[5] = fkj * drq;
    const float sij = (fij + fji) * 0.5f, sik = (fik + fki) * 0.5f, sjk = (fjk + fkj) * 0.5f;
    const float spq = (dpq + dqp) * 0.5f, spr = (dpr + drp) * 0.5f, sqr = (dqr + drq) * 0.5f;
    f[6] = sij;
    f[7] = sik;
    f[8] = sjk;
    f[9] = spq;
    f[10] = spr;
    f[11] = sqr;
    f[12] = T.fa[i];
    f[13] = T.fa[j];
    f[14] = T.fa[k];
    f[15] = T.dl[p];
    f[16] = T.dl[q];
    f[17] = T.dl[r];
    f[18] = T.Xn[i * n + p];
    f[19] = T.Xn[j * n + q];
    f[20] = T.Xn[k * n + r];
    f[21] = T.inv_m;
    f[22] = sij * T.dbar;
    f[23] = sik * T.dbar;
    f[24] = sjk * T.dbar;
    f[25] = spq * T.fbar;
    f[26] = spr * T.fbar;
    f[27] = sqr * T.fbar;
    f[28] = 0.f;
    f[29] = 0.f;
    f[30] = 0.f;
    f[31] = 0.f;
}

// z-array index of member (f1,f2,f3,l1,l2,l3).
__device__ __forceinline__ long long member_index(int n, int f1, int f2, int f3, int l1, int l2, int l3)
{
    const int m = n - 2;
    const long long t = tile_of(n, f1, l1, f2, l2);
    const int row = f3 - (f3 > f1) - (f3 > f2);
    const int col = l3 - (l3 > l1) - (l3 > l2);
    return t * ((long long)m * m) + (long long)row * m + col;
}

// Ids outside [0, total) give rows of NaN.
__global__ void k_orbit_features(const long long *__restrict__ ids, long long count, long long total,
                                 const int *__restrict__ triples, FeatTables T, float *__restrict__ out)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= count) return;
    const long long o = ids[a];
    float f[kFeat];
    if (o >= 0 && o < total) {
        int i, j, k, p, q, r;
        decode_orbit(o, T.n, triples, i, j, k, p, q, r);
        orbit_features(T, i, j, k, p, q, r, f);
    } else {
#pragma unroll
        for (int c = 0; c < kFeat; ++c) f[c] = __builtin_nanf("");
    }
    float4 *dst = (float4 *)(out + a * kFeat);
#pragma unroll
    for (int c = 0; c < kFeat / 4; ++c) dst[c] = make_float4(f[4 * c], f[4 * c + 1], f[4 * c + 2], f[4 * c + 3]);
}

__global__ void k_orbit_targets(const long long *__restrict__ ids, long long count, long long total,
                                const int *__restrict__ triples, int n, const double *__restrict__ Vt, double scale,
                                float *__restrict__ out)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= count) return;
    const long long o = ids[a];
    if (o < 0 || o >= total) {
#pragma unroll
        for (int e = 0; e < kOut; ++e) out[a * kOut + e] = __builtin_nanf("");
        return;
    }
    int i, j, k, p, q, r;
    decode_orbit(o, n, triples, i, j, k, p, q, r);
    const int fac[3] = {i, j, k}, loc[3] = {p, q, r};
    const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const long long z = member_index(n, fac[P[e][0]], fac[P[e][1]], fac[P[e][2]], loc[P[e][0]], loc[P[e][1]],
                                         loc[P[e][2]]);
        out[a * kOut + e] = (float)(Vt[z] / scale);
    }
}

// ------------------------------------------------------- fused inference --
constexpr int kMlpThreads = 512;   // 8 waves, 2 per SIMD
constexpr int kMlpNB = 1;          // 32-orbit column blocks per wave pass (2 spills at 2 waves/SIMD)
constexpr int kOrbitsPerWave = 32 * kMlpNB;

// relu as one integer max on the bit pattern: a negative float (-0 included)
// is a negative int32 and becomes +0, anything else is kept.  fmaxf would add
// a NaN-quieting max first; inputs here are finite.  Plain C, not inline asm:
// the compiler must see this read of MFMA results to insert its wait states.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// Each wave pass takes kMlpNB blocks of 32 orbits; every weight fragment read
// from LDS feeds one MFMA per block.
__global__ __launch_bounds__(kMlpThreads) void k_orbit_mlp(const bf16x8 *__restrict__ Wf,
                                                           const float *__restrict__ master,
                                                           const int *__restrict__ triples, FeatTables T,
                                                           long long count, float *__restrict__ y)
{
    __shared__ bf16x8 wl[kFragTotal];
    __shared__ float bl[2 * kWidth + 8];
    for (int a = threadIdx.x; a < kFragTotal; a += kMlpThreads) wl[a] = Wf[a];
    for (int a = threadIdx.x; a < 2 * kWidth + 8; a += kMlpThreads) {
        float v = 0.f;
        if (a < kWidth)
            v = master[kOffB1 + a];
        else if (a < 2 * kWidth)
            v = master[kOffB2 + a - kWidth];
        else if (a < 2 * kWidth + kOut)
            v = master[kOffB3 + a - 2 * kWidth];
        bl[a] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int w3row = col < kOut ? col : kOut - 1;
    const long long stride = (long long)gridDim.x * (kMlpThreads / 64) * kOrbitsPerWave;
    for (long long base = ((long long)blockIdx.x * (kMlpThreads / 64) + wave) * kOrbitsPerWave; base < count;
         base += stride) {
        // The weight fragments are loop-invariant; an opaque zero offset
        // keeps the compiler from hoisting all of them into registers.
        int z0;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z0));
        const bf16x8 *wv = wl + z0;
        // layer 1 B operands: chunk c of block nb holds inputs 16c + 8h + i
        bf16x8 xb[kMlpNB][2];
#pragma unroll
        for (int nb = 0; nb < kMlpNB; ++nb) {
            const long long o = base + 32 * nb + col;
            float f[kFeat];
            if (o < count) {
                int i, j, k, p, q, r;
                decode_orbit(o, T.n, triples, i, j, k, p, q, r);
                orbit_features(T, i, j, k, p, q, r, f);
            } else {
#pragma unroll
                for (int c = 0; c < kFeat; ++c) f[c] = 0.f;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int i = 0; i < 8; ++i) xb[nb][c][i] = (__bf16)(h ? f[16 * c + 8 + i] : f[16 * c + i]);
        }
        bf16x8 h1[kMlpNB][16];
#pragma unroll
        for (int mb = 0; mb < 8; ++mb) {
            f32x16 acc[kMlpNB];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float b = bl[32 * mb + 8 * (j >> 2) + 4 * h + (j & 3)];
#pragma unroll
                for (int nb = 0; nb < kMlpNB; ++nb) acc[nb][j] = b;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bf16x8 a = wv[kFragW1 + (mb * 2 + c) * 64 + lane];
#pragma unroll
                for (int nb = 0; nb < kMlpNB; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xb[nb][c], acc[nb], 0, 0, 0);
            }
#pragma unroll
            for (int nb = 0; nb < kMlpNB; ++nb)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int i = 0; i < 8; ++i) h1[nb][2 * mb + a][i] = (__bf16)relu(acc[nb][8 * a + i]);
        }
        // layers 2 and 3: each pair of layer-2 output chunks feeds layer 3 at once
        f32x16 acc3[kMlpNB];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = 8 * (j >> 2) + 4 * h + (j & 3);
            const float b = row < kOut ? bl[2 * kWidth + row] : 0.f;
#pragma unroll
            for (int nb = 0; nb < kMlpNB; ++nb) acc3[nb][j] = b;
        }
#pragma unroll
        for (int mb = 0; mb < 8; ++mb) {
            f32x16 acc[kMlpNB];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float b = bl[kWidth + 32 * mb + 8 * (j >> 2) + 4 * h + (j & 3)];
#pragma unroll
                for (int nb = 0; nb < kMlpNB; ++nb) acc[nb][j] = b;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const bf16x8 a = wv[kFragW2 + (mb * 16 + c) * 64 + lane];
#pragma unroll
                for (int nb = 0; nb < kMlpNB; ++nb)
                    acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h1[nb][c], acc[nb], 0, 0, 0);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                bf16x8 w3 = wv[kFragW3 + ((2 * mb + a) * 2 + h) * kOut + w3row];
                if (col >= kOut) w3 = bf16x8{};
#pragma unroll
                for (int nb = 0; nb < kMlpNB; ++nb) {
                    bf16x8 h2;
#pragma unroll
                    for (int i = 0; i < 8; ++i) h2[i] = (__bf16)relu(acc[nb][8 * a + i]);
                    acc3[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w3, h2, acc3[nb], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int nb = 0; nb < kMlpNB; ++nb) {
            const long long o = base + 32 * nb + col;
            if (o < count) {
                float2 *dst = (float2 *)(y + o * kOut);
                if (h == 0) {
                    dst[0] = make_float2(acc3[nb][0], acc3[nb][1]);
                    dst[1] = make_float2(acc3[nb][2], acc3[nb][3]);
                } else {
                    dst[2] = make_float2(acc3[nb][0], acc3[nb][1]);
                }
            }
        }
    }
}

// --------------------------------------------------------- warm z writer --
// Block = one facility triple x one SB^3 cube of locations (the sweep's
// grid).  Orbit phase: one thread per cube cell reads the orbit's six
// outputs, v_e = (y_e - mean) * scale in FP64 (mean a left-to-right sum / 6),
// stages -v_e; store phase writes each member's runs.
__global__ __launch_bounds__(256) void k_warm_z(double *__restrict__ Z, const float *__restrict__ y,
                                                const int *__restrict__ triples, int ntriples, int n, int nb,
                                                double scale)
{
    __shared__ double gs[6 * SB_CUBE];
    const unsigned b = blockIdx.x;
    const unsigned xcd = b & 7u, s = b >> 3;
    const unsigned nb3 = (unsigned)(nb * nb * nb);
    const int tri = (int)((s / nb3) * 8u + xcd);
    if (tri >= ntriples) return;
    const int sub = (int)(s % nb3);
    const int base[3] = {(sub / (nb * nb)) * SB, ((sub / nb) % nb) * SB, (sub % nb) * SB};
    const int packed = triples[tri];
    const int fi = packed & 0xff, fj = (packed >> 8) & 0xff, fk = (packed >> 16) & 0xff;
    const int m = n - 2;
    const long long mm = (long long)m * m;
    const long long L3 = (long long)n * (n - 1) * (n - 2);
    constexpr int PER = (SB * SB * SB) / 256;
#pragma unroll
    for (int w = 0; w < PER; ++w) {
        const int u = threadIdx.x + 256 * w;
        const int rl = u % SB, ql = (u / SB) % SB, pl = u / (SB * SB);
        const int p = base[0] + pl, q = base[1] + ql, r = base[2] + rl;
        if (p < n && q < n && r < n && p != q && p != r && q != r) {
            const int qq = q - (q > p), rr = r - (r > p) - (r > q);
            const long long o = (long long)tri * L3 + ((long long)p * (n - 1) + qq) * (n - 2) + rr;
            const float *yo = y + o * kOut;
            double v[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) v[e] = (double)yo[e];
            const double mean = (((((v[0] + v[1]) + v[2]) + v[3]) + v[4]) + v[5]) / 6.0;
            const int c = cube_idx(pl, ql, rl);
#pragma unroll
            for (int e = 0; e < 6; ++e) gs[e * SB_CUBE + c] = 0.0 - (v[e] - mean) * scale;
        }
    }
    __syncthreads();
    const int F1[6] = {fi, fi, fj, fj, fk, fk};
    const int F2[6] = {fj, fk, fi, fk, fi, fj};
    const int F3[6] = {fk, fj, fk, fi, fj, fi};
    const int X1[6] = {0, 0, 1, 1, 2, 2};
    const int X2[6] = {1, 2, 0, 2, 0, 1};
    const int X3[6] = {2, 1, 2, 0, 1, 0};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
#pragma unroll
        for (int w = 0; w < PER; ++w) {
            const int u = threadIdx.x + 256 * w;
            const int a3 = u % SB, a2 = (u / SB) % SB, a1 = u / (SB * SB);
            int loc[3];
            loc[X1[e]] = base[X1[e]] + a1;
            loc[X2[e]] = base[X2[e]] + a2;
            loc[X3[e]] = base[X3[e]] + a3;
            const int l1 = loc[X1[e]], l2 = loc[X2[e]], l3 = loc[X3[e]];
            if (l1 < n && l2 < n && l3 < n && l1 != l2 && l1 != l3 && l2 != l3) {
                const long long t = tile_of(n, F1[e], l1, F2[e], l2);
                const int row = F3[e] - (F3[e] > F1[e]) - (F3[e] > F2[e]);
                const int col = l3 - (l3 > l1) - (l3 > l2);
                Z[t * mm + (long long)row * m + col] =
                    gs[e * SB_CUBE + cube_idx(loc[0] - base[0], loc[1] - base[1], loc[2] - base[2])];
            }
        }
    }
}

// Element-wise helpers of the S-form restart.
__global__ void k_negate(double *__restrict__ a, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) a[i] = 0.0 - a[i];
}

__global__ void k_sub(double *__restrict__ a, const double *__restrict__ b, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) a[i] = a[i] - b[i];
}

// ---------------------------------------------------------- training GEMM --
// C(m,n) = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) =
// B[k*sbk + n*sbn]; operands rounded to bf16 on their way into LDS, fp32
// accumulation.  64x64 tile per block, 2x2 waves of 32x32, K step 16.
enum GemmEpi { kEpiStore = 0, kEpiBiasRelu = 1, kEpiBias = 2, kEpiMask = 3 };

struct GemmOut {
    float *c;            // fp32 output (kEpiStore, kEpiBias; kEpiMask: unrounded product)
    __bf16 *cb;          // bf16 output (kEpiBiasRelu, kEpiMask)
    long long ldc;       // row pitch of both outputs
    const float *bias;   // per row m
    const __bf16 *mask;  // kEpiMask: keep where mask(m,n) > 0, pitch ldc
};

constexpr int kGemmKP = 24;  // LDS pitch of one 16-wide K slice (bf16), keeps rows 16-byte aligned

__device__ __forceinline__ float load_f(const float *p) { return *p; }
__device__ __forceinline__ float load_f(const __bf16 *p) { return (float)*p; }

template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const TA *__restrict__ A, long long sam, long long sak,
                                              const TB *__restrict__ B, long long sbk, long long sbn, int M, int N,
                                              int K, GemmOut out)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[64 * kGemmKP];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[64 * kGemmKP];
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, col = lane & 31;
    const int lr = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 4;  // loader: row/col lr, 4 k from lk
    f32x16 acc = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int k = k0 + lk + d;
            const int mA = m0 + lr, nB = n0 + lr;
            const float a = (mA < M && k < K) ? load_f(A + mA * sam + k * sak) : 0.f;
            const float bv = (nB < N && k < K) ? load_f(B + k * sbk + nB * sbn) : 0.f;
            As[lr * kGemmKP + lk + d] = (__bf16)a;
            Bs[lr * kGemmKP + lk + d] = (__bf16)bv;
        }
        __syncthreads();
        const bf16x8 af = *(const bf16x8 *)(As + (wm * 32 + col) * kGemmKP + 8 * h);
        const bf16x8 bf = *(const bf16x8 *)(Bs + (wn * 32 + col) * kGemmKP + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, acc, 0, 0, 0);
        __syncthreads();
    }
    const int n = n0 + wn * 32 + col;
    if (n >= N) return;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int m = m0 + wm * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
        if (m >= M) continue;
        const long long at = (long long)m * out.ldc + n;
        float v = acc[j];
        if (EPI == kEpiStore) {
            out.c[at] = v;
        } else if (EPI == kEpiBias) {
            out.c[at] = v + out.bias[m];
        } else if (EPI == kEpiBiasRelu) {
            out.cb[at] = (__bf16)fmaxf(v + out.bias[m], 0.f);
        } else {
            v = ((float)out.mask[at] > 0.f) ? v : 0.f;
            out.c[at] = v;
            out.cb[at] = (__bf16)v;
        }
    }
}

// Output error of the projected MSE loss, per sample b (column of Y):
// yh = y - mean(y); g = 2 (yh - t) / (6 N); delta3 = g - mean(g).  Writes
// delta3 as fp32 and bf16 ([6][N]) and one partial sum of (yh - t)^2 per block.
__global__ __launch_bounds__(256) void k_out_err(const float *__restrict__ Y, const float *__restrict__ Tg, int N,
                                                 float *__restrict__ d3f, __bf16 *__restrict__ d3b,
                                                 double *__restrict__ part)
{
    __shared__ double red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double se = 0.0;
    if (b < N) {
        float y[kOut], g[kOut];
        float s = 0.f;
#pragma unroll
        for (int e = 0; e < kOut; ++e) {
            y[e] = Y[(long long)e * N + b];
            s += y[e];
        }
        const float mean = s / 6.f;
        const float inv = 2.f / (6.f * (float)N);
        float gs = 0.f;
#pragma unroll
        for (int e = 0; e < kOut; ++e) {
            const float d = (y[e] - mean) - Tg[(long long)b * kOut + e];
            se += (double)d * (double)d;
            g[e] = d * inv;
            gs += g[e];
        }
        const float gm = gs / 6.f;
#pragma unroll
        for (int e = 0; e < kOut; ++e) {
            const float d3 = g[e] - gm;
            d3f[(long long)e * N + b] = d3;
            d3b[(long long)e * N + b] = (__bf16)d3;
        }
    }
    red[threadIdx.x] = se;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[m] = sum_n D[m*N + n], fixed order (one block per row).
__global__ __launch_bounds__(256) void k_rowsum(const float *__restrict__ Dm, int N, float *__restrict__ out)
{
    __shared__ float red[256];
    const int m = blockIdx.x;
    float s = 0.f;
    for (int n = threadIdx.x; n < N; n += 256) s += Dm[(long long)m * N + n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[m] = red[0];
}

// y[b][e] = Y[e][b] (the caller's sample-major layout).
__global__ void k_out_transpose(const float *__restrict__ Y, int N, float *__restrict__ y)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N * kOut) return;
    const int b = a / kOut, e = a % kOut;
    y[a] = Y[(long long)e * N + b];
}

// Adam (Kingma and Ba) on the float32 masters; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ mo,
                       float *__restrict__ vo, int count, float lr, float beta1, float beta2, float eps, float bc1,
                       float bc2)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= count) return;
    const float gg = g[a];
    const float m = beta1 * mo[a] + (1.f - beta1) * gg;
    const float v = beta2 * vo[a] + (1.f - beta2) * gg * gg;
    mo[a] = m;
    vo[a] = v;
    const float mh = m / bc1, vh = v / bc2;
    w[a] = w[a] - lr * mh / (sqrtf(vh) + eps);
}

// bf16 copies of the weights: row-major (GEMMs) and MFMA fragments.
__global__ void k_mlp_pack(const float *__restrict__ master, __bf16 *__restrict__ rowc, bf16x8 *__restrict__ frag)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < kRowTotal) {
        const int src = a < kRowW2 ? kOffW1 + a : a < kRowW3 ? kOffW2 + (a - kRowW2) : kOffW3 + (a - kRowW3);
        rowc[a] = (__bf16)master[src];
    }
    if (a < kFragTotal) {
        bf16x8 v;
        if (a < kFragW2) {  // [mb][c][lane]: W1[32 mb + lane%32][16 c + 8 (lane/32) + i]
            const int lane = a & 63, c = (a >> 6) & 1, mb = a >> 7;
            const int row = 32 * mb + (lane & 31);
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (__bf16)master[kOffW1 + row * kFeat + 16 * c + 8 * (lane >> 5) + i];
        } else if (a < kFragW3) {  // [mb][c][lane]: W2[32 mb + lane%32][chunk_feature(c, lane/32, i)]
            const int b = a - kFragW2;
            const int lane = b & 63, c = (b >> 6) & 15, mb = b >> 10;
            const int row = 32 * mb + (lane & 31);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                v[i] = (__bf16)master[kOffW2 + row * kWidth + chunk_feature(c, lane >> 5, i)];
        } else {  // [c][half][row]: W3[row][chunk_feature(c, half, i)]
            const int b = a - kFragW3;
            const int row = b % kOut, half = (b / kOut) & 1, c = b / (2 * kOut);
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (__bf16)master[kOffW3 + row * kWidth + chunk_feature(c, half, i)];
        }
        frag[a] = v;
    }
}

}  // namespace qap
