// learn_host.hpp -- host side of multiplier tracking, the S-form restart and
// the learned warm start (included at the end of capi.hip: one translation
// unit with the context helpers).
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

#include "learn.hpp"

struct qap_mlp {
    hipStream_t stream = nullptr;
    int max_batch = 0;
    int step = 0;  // Adam steps taken
    void *arena = nullptr;
    float *master = nullptr, *grad = nullptr, *mom1 = nullptr, *mom2 = nullptr;
    __bf16 *rowc = nullptr;  // row-major bf16 copies
    bf16x8 *frag = nullptr;  // MFMA fragment copies
    // training activations for up to max_batch samples, feature-major
    __bf16 *H1 = nullptr, *H2 = nullptr, *D1b = nullptr, *D2b = nullptr, *D3b = nullptr;
    float *Y = nullptr, *D1f = nullptr, *D2f = nullptr, *D3f = nullptr;
    double *part = nullptr;
    int cu = 256;  // compute units of the device (persistent grid)
    std::string err;
};

namespace {

int mfail(qap_mlp *p, int code, const std::string &msg)
{
    if (p)
        p->err = msg;
    else
        g_init_error = msg;
    return code;
}

#define MHIPCHK(p, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return mfail((p), QAP_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));  \
    } while (0)

void *dev_alloc(qap_ctx *h, size_t bytes)
{
    void *p = nullptr;
    if (h->prm.alloc) return h->prm.alloc(bytes, h->prm.alloc_ctx);
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(qap_ctx *h, void *p)
{
    if (!p) return;
    if (h->prm.alloc) {
        if (h->prm.free_fn) h->prm.free_fn(p, h->prm.alloc_ctx);
    } else {
        (void)hipFree(p);
    }
}

unsigned fill_blocks(size_t count) { return (unsigned)std::min<size_t>((count + 255) / 256, 16384); }

// Zero the tracking arrays (if tracking).
hipError_t zero_tracking(qap_ctx *h)
{
    if (!h->Vt) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(h->Vz)), dim3(256), 0, h->stream, h->Vt, h->Vz, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks((size_t)h->T)), dim3(256), 0, h->stream, h->Ut, (size_t)h->T, 0.0);
    return hipGetLastError();
}

// Algorithm 1 step 1 for the x and y levels (x costs b + f_ii d_pp, y costs
// C), pi arrays cleared; the z array is the caller's.
hipError_t reset_xy(qap_ctx *h)
{
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks((size_t)h->T)), dim3(256), 0, h->stream, h->Py, (size_t)h->T, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->stream, h->Px, (size_t)h->n * h->n, 0.0);
    hipLaunchKernelGGL(k_init_xy, dim3(std::min<long long>((h->T + 255) / 256, 65535)), dim3(256), 0, h->stream,
                       h->F, h->D, h->B, h->Xc, h->Yc, h->n);
    return hipGetLastError();
}

// Compact indices of the six members of orbit (i,j,k,p,q,r), canonical order.
void orbit_members_host(int n, int i, int j, int k, int p, int q, int r, size_t out[6])
{
    const int fac[3] = {i, j, k}, loc[3] = {p, q, r};
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int m = n - 2;
    for (int e = 0; e < 6; ++e) {
        const int f1 = fac[P[e][0]], f2 = fac[P[e][1]], f3 = fac[P[e][2]];
        const int l1 = loc[P[e][0]], l2 = loc[P[e][1]], l3 = loc[P[e][2]];
        const size_t t = (((size_t)(f1 * n + l1) * (n - 1) + (f2 - (f2 > f1))) * (n - 1) + (l2 - (l2 > l1)));
        out[e] = t * (size_t)m * m + (size_t)(f3 - (f3 > f1) - (f3 > f2)) * m + (size_t)(l3 - (l3 > l1) - (l3 > l2));
    }
}

// Per-instance feature tables (float32, computed in FP64) and the multiplier
// scale s / (n - 2), s = max(1, max|F|) * max(1, max|D|).
struct HostTables {
    std::vector<float> buf;  // Fn, Dn, Xn (n*n each), fa, dl (n each)
    float fbar = 0, dbar = 0, inv_m = 0;
    double scale = 1.0;
};

HostTables host_tables(const qap_ctx *h)
{
    const int n = h->n;
    const double *F = h->hF.data(), *D = h->hD.data(), *B = h->hB.data();
    double sF = 1.0, sD = 1.0;
    for (int a = 0; a < n * n; ++a) {
        sF = std::fmax(sF, std::fabs(F[a]));
        sD = std::fmax(sD, std::fabs(D[a]));
    }
    HostTables t;
    t.scale = sF * sD / (double)(n - 2);
    t.buf.assign((size_t)3 * n * n + 2 * n, 0.f);
    float *Fn = t.buf.data(), *Dn = Fn + n * n, *Xn = Dn + n * n, *fa = Xn + n * n, *dl = fa + n;
    double fsum = 0.0, dsum = 0.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            Fn[a * n + b] = (float)(F[a * n + b] / sF);
            Dn[a * n + b] = (float)(D[a * n + b] / sD);
            Xn[a * n + b] = (float)((B[a * n + b] + F[a * n + a] * D[b * n + b]) / (sF * sD));
            if (a != b) {
                fsum += F[a * n + b] / sF;
                dsum += D[a * n + b] / sD;
            }
        }
    for (int a = 0; a < n; ++a) {
        double fr = 0.0, dr = 0.0;
        for (int l = 0; l < n; ++l) {
            fr += F[a * n + l] / sF + F[l * n + a] / sF;
            dr += D[a * n + l] / sD + D[l * n + a] / sD;
        }
        fa[a] = (float)(fr / (2.0 * n));
        dl[a] = (float)(dr / (2.0 * n));
    }
    t.fbar = (float)(fsum / ((double)n * (n - 1)));
    t.dbar = (float)(dsum / ((double)n * (n - 1)));
    t.inv_m = (float)(1.0 / (double)(n - 2));
    return t;
}

// Upload the tables into a fresh device buffer; returns the descriptor.
int upload_tables(qap_ctx *h, const HostTables &t, float **dev, FeatTables &ft)
{
    const int n = h->n;
    *dev = (float *)dev_alloc(h, sizeof(float) * t.buf.size());
    if (!*dev) return fail(h, QAP_ENOMEM, "feature table allocation failed");
    HIPCHK(h, hipMemcpyAsync(*dev, t.buf.data(), sizeof(float) * t.buf.size(), hipMemcpyHostToDevice, h->stream));
    ft.Fn = *dev;
    ft.Dn = ft.Fn + n * n;
    ft.Xn = ft.Dn + n * n;
    ft.fa = ft.Xn + n * n;
    ft.dl = ft.fa + n;
    ft.fbar = t.fbar;
    ft.dbar = t.dbar;
    ft.inv_m = t.inv_m;
    ft.n = n;
    return QAP_OK;
}

long long orbit_count_of(int n) { return (long long)n * (n - 1) * (n - 2) / 6 * ((long long)n * (n - 1) * (n - 2)); }

// Restart in S-form with z costs already in h->Z: x/y costs of step 1, LB 0, t 0.
int restart_s_form(qap_ctx *h)
{
    hipError_t e = reset_xy(h);
    if (e != hipSuccess) return fail(h, QAP_EDEVICE, std::string("restart: ") + hipGetErrorString(e));
    if ((e = zero_tracking(h)) != hipSuccess) return fail(h, QAP_EDEVICE, hipGetErrorString(e));
    return upload_scalars(h, 0.0);
}

int mlp_pack(qap_mlp *p)
{
    const int cnt = std::max(kRowTotal, kFragTotal);
    hipLaunchKernelGGL(k_mlp_pack, dim3((cnt + 255) / 256), dim3(256), 0, p->stream, p->master, p->rowc, p->frag);
    MHIPCHK(p, hipGetLastError());
    return QAP_OK;
}

template <typename TA, typename TB, int EPI>
hipError_t gemm(hipStream_t s, const TA *A, long long sam, long long sak, const TB *B, long long sbk, long long sbn,
                int M, int N, int K, GemmOut o)
{
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, K, o);
    return hipGetLastError();
}

// Forward of the training path over N samples (features x: [N][32] fp32):
// H1, H2 (bf16, [256][N]) and Y (fp32, [6][N]).
hipError_t mlp_forward_gemm(qap_mlp *p, const float *x, int N)
{
    hipError_t e;
    const __bf16 *W1 = p->rowc + kRowW1, *W2 = p->rowc + kRowW2, *W3 = p->rowc + kRowW3;
    GemmOut o{};
    o.ldc = N;
    o.cb = p->H1;
    o.bias = p->master + kOffB1;
    if ((e = gemm<__bf16, float, kEpiBiasRelu>(p->stream, W1, kFeat, 1, x, 1, kFeat, kWidth, N, kFeat, o)) != hipSuccess)
        return e;
    o.cb = p->H2;
    o.bias = p->master + kOffB2;
    if ((e = gemm<__bf16, __bf16, kEpiBiasRelu>(p->stream, W2, kWidth, 1, p->H1, N, 1, kWidth, N, kWidth, o)) !=
        hipSuccess)
        return e;
    o.cb = nullptr;
    o.c = p->Y;
    o.bias = p->master + kOffB3;
    return gemm<__bf16, __bf16, kEpiBias>(p->stream, W3, kWidth, 1, p->H2, N, 1, kOut, N, kWidth, o);
}

// Gradients of the projected MSE loss into p->grad; loss to *loss.
int mlp_backward(qap_mlp *p, const float *x, const float *t, int N, double *loss)
{
    hipError_t e;
    if ((e = mlp_forward_gemm(p, x, N)) != hipSuccess) return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    const int eb = (N + 255) / 256;
    hipLaunchKernelGGL(k_out_err, dim3(eb), dim3(256), 0, p->stream, p->Y, t, N, p->D3f, p->D3b, p->part);
    const __bf16 *W2 = p->rowc + kRowW2, *W3 = p->rowc + kRowW3;
    GemmOut o{};
    // dW3[o][f] = sum_b d3(o,b) h2(f,b)
    o.c = p->grad + kOffW3;
    o.ldc = kWidth;
    if ((e = gemm<__bf16, __bf16, kEpiStore>(p->stream, p->D3b, N, 1, p->H2, 1, N, kOut, kWidth, N, o)) != hipSuccess)
        return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    // delta2[f][b] = (sum_o W3[o][f] d3(o,b)) masked by h2 > 0
    o = GemmOut{};
    o.c = p->D2f;
    o.cb = p->D2b;
    o.ldc = N;
    o.mask = p->H2;
    if ((e = gemm<__bf16, __bf16, kEpiMask>(p->stream, W3, 1, kWidth, p->D3b, N, 1, kWidth, N, kOut, o)) != hipSuccess)
        return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    // dW2[o][i] = sum_b d2(o,b) h1(i,b)
    o = GemmOut{};
    o.c = p->grad + kOffW2;
    o.ldc = kWidth;
    if ((e = gemm<__bf16, __bf16, kEpiStore>(p->stream, p->D2b, N, 1, p->H1, 1, N, kWidth, kWidth, N, o)) !=
        hipSuccess)
        return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    // delta1[i][b] = (sum_o W2[o][i] d2(o,b)) masked by h1 > 0
    o = GemmOut{};
    o.c = p->D1f;
    o.cb = p->D1b;
    o.ldc = N;
    o.mask = p->H1;
    if ((e = gemm<__bf16, __bf16, kEpiMask>(p->stream, W2, 1, kWidth, p->D2b, N, 1, kWidth, N, kWidth, o)) !=
        hipSuccess)
        return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    // dW1[i][f] = sum_b d1(i,b) x(b,f)
    o = GemmOut{};
    o.c = p->grad + kOffW1;
    o.ldc = kFeat;
    if ((e = gemm<__bf16, float, kEpiStore>(p->stream, p->D1b, N, 1, x, kFeat, 1, kWidth, kFeat, N, o)) != hipSuccess)
        return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    hipLaunchKernelGGL(k_rowsum, dim3(kWidth), dim3(256), 0, p->stream, p->D1f, N, p->grad + kOffB1);
    hipLaunchKernelGGL(k_rowsum, dim3(kWidth), dim3(256), 0, p->stream, p->D2f, N, p->grad + kOffB2);
    hipLaunchKernelGGL(k_rowsum, dim3(kOut), dim3(256), 0, p->stream, p->D3f, N, p->grad + kOffB3);
    MHIPCHK(p, hipGetLastError());
    if (loss) {
        std::vector<double> part(eb);
        MHIPCHK(p, hipMemcpyAsync(part.data(), p->part, sizeof(double) * eb, hipMemcpyDeviceToHost, p->stream));
        MHIPCHK(p, hipStreamSynchronize(p->stream));
        double s = 0.0;
        for (double v : part) s += v;
        *loss = s / (6.0 * N);
    }
    return QAP_OK;
}

}  // namespace

extern "C" {

int qap_track(qap_handle h, int on)
{
    if (!h) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "multiplier tracking follows the FULL shares");
    if (h->prm.two_phase && !h->prm.slow)
        return fail(h, QAP_EUNSUPPORTED, "multiplier tracking does not follow the F2 pooling");
    if (h->sa_on && on) return fail(h, QAP_EUNSUPPORTED, "multiplier tracking does not follow Type 4 steps");
    if (h->prm.slow && !on) return fail(h, QAP_EUNSUPPORTED, "an S1 handle keeps its multipliers tracked");
    if (h->prm.slow && h->Vt) return QAP_OK;  // already on: its multipliers are the S1 state, keep them
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (!on) {
        dev_free(h, h->Vt);
        dev_free(h, h->Ut);
        h->Vt = h->Ut = nullptr;
    } else if (!h->Vt) {
        h->Vt = (double *)dev_alloc(h, sizeof(double) * h->Vz);
        h->Ut = (double *)dev_alloc(h, sizeof(double) * (size_t)h->T);
        if (!h->Vt || !h->Ut) {
            dev_free(h, h->Vt);
            dev_free(h, h->Ut);
            h->Vt = h->Ut = nullptr;
            return fail(h, QAP_ENOMEM, "tracking arrays do not fit in device memory");
        }
    }
    hipError_t e = zero_tracking(h);
    if (e != hipSuccess) return fail(h, QAP_EDEVICE, hipGetErrorString(e));
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return QAP_OK;
}

int qap_set_allocator(qap_handle h, qap_alloc_fn alloc, qap_free_fn free_fn, void *ctx)
{
    if (!h) return QAP_EINVAL;
    if (alloc && !free_fn) return fail(h, QAP_EINVAL, "an allocator needs a free function");
    if (h->Vt) return fail(h, QAP_ESTATE, "tracking arrays are live (qap_track(h, 0) first)");
    h->prm.alloc = alloc;
    h->prm.free_fn = free_fn;
    h->prm.alloc_ctx = ctx;
    return QAP_OK;
}

int qap_get_multipliers(qap_handle h, double *v, double *u)
{
    if (!h) return QAP_EINVAL;
    if (!h->Vt) return fail(h, QAP_ESTATE, "multiplier tracking is off (qap_track)");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (v) HIPCHK(h, hipMemcpy(v, h->Vt, sizeof(double) * h->Vz, hipMemcpyDeviceToHost));
    if (u) HIPCHK(h, hipMemcpy(u, h->Ut, sizeof(double) * (size_t)h->T, hipMemcpyDeviceToHost));
    return QAP_OK;
}

int qap_set_multipliers(qap_handle h, const double *v, const double *u)
{
    if (!h) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "z multipliers are FULL-scheme only");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "an S1 handle sets its own multipliers");
    const int n = h->n;
    // zero sums: every orbit of v, every y pair of u
    if (v) {
        double vmax = 0.0;
        for (size_t a = 0; a < h->Vz; ++a) {
            if (!std::isfinite(v[a])) return fail(h, QAP_EINVAL, "non-finite multiplier");
            vmax = std::fmax(vmax, std::fabs(v[a]));
        }
        const double tol = 1e-9 * std::fmax(1.0, vmax);
        size_t idx[6];
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                for (int k = j + 1; k < n; ++k)
                    for (int p = 0; p < n; ++p)
                        for (int q = 0; q < n; ++q) {
                            if (q == p) continue;
                            for (int r = 0; r < n; ++r) {
                                if (r == p || r == q) continue;
                                orbit_members_host(n, i, j, k, p, q, r, idx);
                                double s = 0.0;
                                for (int e = 0; e < 6; ++e) s += v[idx[e]];
                                if (std::fabs(s) > tol)
                                    return fail(h, QAP_EINVAL, "z multipliers do not sum to zero over an orbit");
                            }
                        }
    }
    if (u) {
        double umax = 0.0;
        for (long long a = 0; a < h->T; ++a) {
            if (!std::isfinite(u[a])) return fail(h, QAP_EINVAL, "non-finite multiplier");
            umax = std::fmax(umax, std::fabs(u[a]));
        }
        const double tol = 1e-9 * std::fmax(1.0, umax);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q) {
                        if (q == p) continue;
                        const size_t a = ((size_t)(i * n + p) * (n - 1) + (j - (j > i))) * (n - 1) + (q - (q > p));
                        const size_t b = ((size_t)(j * n + q) * (n - 1) + (i - (i > j))) * (n - 1) + (p - (p > q));
                        if (std::fabs(u[a] + u[b]) > tol)
                            return fail(h, QAP_EINVAL, "y multipliers do not sum to zero over a pair");
                    }
            }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (v) {
        HIPCHK(h, hipMemcpy(h->Z, v, sizeof(double) * h->Vz, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_negate, dim3(fill_blocks(h->Vz)), dim3(256), 0, h->stream, h->Z, h->Vz);
    } else {
        hipLaunchKernelGGL(k_fill, dim3(fill_blocks(h->Vz)), dim3(256), 0, h->stream, h->Z, h->Vz, 0.0);
    }
    HIPCHK(h, hipGetLastError());
    hipError_t e = reset_xy(h);
    if (e != hipSuccess) return fail(h, QAP_EDEVICE, hipGetErrorString(e));
    if (u) {
        // Yc <- C - u, staged through Py (cleared again afterwards)
        HIPCHK(h, hipStreamSynchronize(h->stream));
        HIPCHK(h, hipMemcpy(h->Py, u, sizeof(double) * (size_t)h->T, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_sub, dim3(fill_blocks((size_t)h->T)), dim3(256), 0, h->stream, h->Yc, h->Py,
                           (size_t)h->T);
        hipLaunchKernelGGL(k_fill, dim3(fill_blocks((size_t)h->T)), dim3(256), 0, h->stream, h->Py, (size_t)h->T,
                           0.0);
        HIPCHK(h, hipGetLastError());
    }
    if ((e = zero_tracking(h)) != hipSuccess) return fail(h, QAP_EDEVICE, hipGetErrorString(e));
    return upload_scalars(h, 0.0);
}

int qap_orbit_count(int n, int64_t *count)
{
    if (!count || n < 3 || n > 64) return fail(nullptr, QAP_EINVAL, "n must be in 3..64");
    *count = orbit_count_of(n);
    return QAP_OK;
}

int qap_multiplier_scale(qap_handle h, double *scale)
{
    if (!h || !scale) return QAP_EINVAL;
    *scale = host_tables(h).scale;
    return QAP_OK;
}

int qap_orbit_features(qap_handle h, const int64_t *ids, int64_t count, float *x)
{
    if (!h || count < 0 || (count > 0 && (!ids || !x))) return QAP_EINVAL;
    if (count == 0) return QAP_OK;
    HostTables t = host_tables(h);
    float *tab = nullptr;
    FeatTables ft{};
    int rc = upload_tables(h, t, &tab, ft);
    if (rc != QAP_OK) return rc;
    hipLaunchKernelGGL(k_orbit_features, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, h->stream,
                       (const long long *)ids, (long long)count, orbit_count_of(h->n), h->triples, ft, x);
    hipError_t e = hipGetLastError();
    hipError_t s = hipStreamSynchronize(h->stream);
    dev_free(h, tab);
    if (e != hipSuccess || s != hipSuccess)
        return fail(h, QAP_EDEVICE, hipGetErrorString(e != hipSuccess ? e : s));
    return QAP_OK;
}

int qap_orbit_targets(qap_handle h, const int64_t *ids, int64_t count, double scale, float *t)
{
    if (!h || count < 0 || (count > 0 && (!ids || !t)) || !(scale > 0.0)) return QAP_EINVAL;
    if (!h->Vt) return fail(h, QAP_ESTATE, "multiplier tracking is off (qap_track)");
    if (count == 0) return QAP_OK;
    hipLaunchKernelGGL(k_orbit_targets, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, h->stream,
                       (const long long *)ids, (long long)count, orbit_count_of(h->n), h->triples, h->n, h->Vt,
                       scale, t);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return QAP_OK;
}

int qap_warm_start_outputs(qap_handle h, const float *y, double scale)
{
    if (!h || !y || !(scale > 0.0) || !std::isfinite(scale)) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "warm starts are FULL-scheme only");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "warm starts are F-form only");
    const int nb = (h->n + SB - 1) / SB;
    const unsigned groups8 = (unsigned)((h->ntriples + 7) / 8);
    const unsigned blocks = groups8 * 8u * (unsigned)(nb * nb * nb);
    hipLaunchKernelGGL(k_warm_z, dim3(blocks), dim3(256), 0, h->stream, h->Z, y, h->triples, h->ntriples, h->n, nb,
                       scale);
    HIPCHK(h, hipGetLastError());
    return restart_s_form(h);
}

// ------------------------------------------------------------- the MLP --
int qap_mlp_create(const float *params, int max_batch, void *stream, qap_mlp_handle *out)
{
    if (!params || !out || max_batch < 1 || max_batch > (1 << 22))
        return mfail(nullptr, QAP_EINVAL, "params/out required, max_batch in 1..2^22");
    for (int a = 0; a < kParams; ++a)
        if (!std::isfinite(params[a])) return mfail(nullptr, QAP_EINVAL, "non-finite parameter");
    qap_mlp *p = new qap_mlp();
    p->stream = (hipStream_t)stream;
    p->max_batch = max_batch;
    const size_t N = (size_t)max_batch;
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t fbytes = r(sizeof(float) * kParams);
    const size_t bytes = 4 * fbytes + r(sizeof(__bf16) * kRowTotal) + r(sizeof(bf16x8) * kFragTotal) +
                         4 * r(sizeof(__bf16) * kWidth * N) + r(sizeof(__bf16) * kOut * N) +
                         r(sizeof(float) * kOut * N) * 2 + 2 * r(sizeof(float) * kWidth * N) +
                         r(sizeof(double) * ((N + 255) / 256));
    if (hipMalloc(&p->arena, bytes) != hipSuccess) {
        delete p;
        return mfail(nullptr, QAP_ENOMEM, "perceptron arena allocation failed");
    }
    char *c = (char *)p->arena;
    auto take = [&](size_t b) {
        char *q = c;
        c += r(b);
        return (void *)q;
    };
    p->master = (float *)take(sizeof(float) * kParams);
    p->grad = (float *)take(sizeof(float) * kParams);
    p->mom1 = (float *)take(sizeof(float) * kParams);
    p->mom2 = (float *)take(sizeof(float) * kParams);
    p->rowc = (__bf16 *)take(sizeof(__bf16) * kRowTotal);
    p->frag = (bf16x8 *)take(sizeof(bf16x8) * kFragTotal);
    p->H1 = (__bf16 *)take(sizeof(__bf16) * kWidth * N);
    p->H2 = (__bf16 *)take(sizeof(__bf16) * kWidth * N);
    p->D1b = (__bf16 *)take(sizeof(__bf16) * kWidth * N);
    p->D2b = (__bf16 *)take(sizeof(__bf16) * kWidth * N);
    p->D3b = (__bf16 *)take(sizeof(__bf16) * kOut * N);
    p->Y = (float *)take(sizeof(float) * kOut * N);
    p->D3f = (float *)take(sizeof(float) * kOut * N);
    p->D1f = (float *)take(sizeof(float) * kWidth * N);
    p->D2f = (float *)take(sizeof(float) * kWidth * N);
    p->part = (double *)take(sizeof(double) * ((N + 255) / 256));
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        p->cu = prop.multiProcessorCount;
    auto cleanup = [&](int code) {
        const std::string e = p->err;
        qap_mlp_destroy(p);
        g_init_error = e;
        return code;
    };
    if (hipMemcpyAsync(p->master, params, sizeof(float) * kParams, hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return cleanup(mfail(p, QAP_EDEVICE, "parameter upload failed"));
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(kParams)), dim3(256), 0, p->stream, (double *)p->mom1,
                       (size_t)(2 * fbytes / sizeof(double)), 0.0);
    int rc = mlp_pack(p);
    if (rc != QAP_OK) return cleanup(rc);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return cleanup(mfail(p, QAP_EDEVICE, "stream error"));
    *out = p;
    return QAP_OK;
}

int qap_mlp_destroy(qap_mlp_handle p)
{
    if (!p) return QAP_EINVAL;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    (void)hipDeviceSynchronize();
    if (p->arena) (void)hipFree(p->arena);
    delete p;
    return QAP_OK;
}

int qap_mlp_set_stream(qap_mlp_handle p, void *stream)
{
    if (!p) return QAP_EINVAL;
    MHIPCHK(p, hipStreamSynchronize(p->stream));
    p->stream = (hipStream_t)stream;
    return QAP_OK;
}

int qap_mlp_get_params(qap_mlp_handle p, float *params)
{
    if (!p || !params) return QAP_EINVAL;
    MHIPCHK(p, hipMemcpyAsync(params, p->master, sizeof(float) * kParams, hipMemcpyDeviceToHost, p->stream));
    MHIPCHK(p, hipStreamSynchronize(p->stream));
    return QAP_OK;
}

int qap_mlp_forward(qap_mlp_handle p, const float *x, int count, float *y)
{
    if (!p || count < 0 || count > p->max_batch || (count > 0 && (!x || !y)))
        return mfail(p, QAP_EINVAL, "count must be in 0..max_batch");
    if (count == 0) return QAP_OK;
    hipError_t e = mlp_forward_gemm(p, x, count);
    if (e != hipSuccess) return mfail(p, QAP_EDEVICE, hipGetErrorString(e));
    // Y is [6][count]; the caller's layout is [count][6]
    hipLaunchKernelGGL(k_out_transpose, dim3((count * kOut + 255) / 256), dim3(256), 0, p->stream, p->Y, count, y);
    MHIPCHK(p, hipGetLastError());
    return QAP_OK;
}

int qap_mlp_gradients(qap_mlp_handle p, const float *x, const float *t, int count, float *grad, double *loss)
{
    if (!p || count < 1 || count > p->max_batch || !x || !t) return mfail(p, QAP_EINVAL, "count must be in 1..max_batch");
    int rc = mlp_backward(p, x, t, count, loss);
    if (rc != QAP_OK) return rc;
    if (grad) {
        MHIPCHK(p, hipMemcpyAsync(grad, p->grad, sizeof(float) * kParams, hipMemcpyDeviceToHost, p->stream));
        MHIPCHK(p, hipStreamSynchronize(p->stream));
    }
    return QAP_OK;
}

int qap_mlp_train_step(qap_mlp_handle p, const float *x, const float *t, int count, const qap_adam_params *opt,
                       double *loss)
{
    if (!p || !opt || count < 1 || count > p->max_batch || !x || !t)
        return mfail(p, QAP_EINVAL, "count must be in 1..max_batch");
    if (!(opt->lr > 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) || !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) ||
        !(opt->eps > 0.0))
        return mfail(p, QAP_EINVAL, "bad Adam hyper-parameters");
    int rc = mlp_backward(p, x, t, count, loss);
    if (rc != QAP_OK) return rc;
    p->step += 1;
    const double bc1 = 1.0 - std::pow(opt->beta1, p->step), bc2 = 1.0 - std::pow(opt->beta2, p->step);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, p->stream, p->master, p->grad, p->mom1,
                       p->mom2, kParams, (float)opt->lr, (float)opt->beta1, (float)opt->beta2, (float)opt->eps,
                       (float)bc1, (float)bc2);
    MHIPCHK(p, hipGetLastError());
    return mlp_pack(p);
}

int qap_orbit_outputs(qap_handle h, qap_mlp_handle p, float *y)
{
    if (!h || !p || !y) return QAP_EINVAL;
    HostTables t = host_tables(h);
    float *tab = nullptr;
    FeatTables ft{};
    int rc = upload_tables(h, t, &tab, ft);
    if (rc != QAP_OK) return rc;
    // the perceptron's copies are written on its stream
    HIPCHK(h, hipStreamSynchronize(p->stream));
    const long long count = orbit_count_of(h->n);
    hipLaunchKernelGGL(k_orbit_mlp, dim3((unsigned)p->cu), dim3(kMlpThreads), 0, h->stream, p->frag, p->master,
                       h->triples, ft, count, y);
    hipError_t e = hipGetLastError();
    hipError_t s = hipStreamSynchronize(h->stream);
    dev_free(h, tab);
    if (e != hipSuccess || s != hipSuccess) return fail(h, QAP_EDEVICE, hipGetErrorString(e != hipSuccess ? e : s));
    return QAP_OK;
}

int qap_warm_start(qap_handle h, qap_mlp_handle p, double gain, qap_warm_stats *st)
{
    if (!h || !p) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "warm starts are FULL-scheme only");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "warm starts are F-form only");
    if (!(gain > 0.0) || !std::isfinite(gain)) return fail(h, QAP_EINVAL, "gain must be positive and finite");
    auto t0 = std::chrono::steady_clock::now();
    const long long count = orbit_count_of(h->n);
    float *y = (float *)dev_alloc(h, sizeof(float) * kOut * (size_t)count);
    if (!y) return fail(h, QAP_ENOMEM, "orbit output buffer does not fit in device memory");
    hipEvent_t ev[3];
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            dev_free(h, y);
            return fail(h, QAP_EDEVICE, "event creation failed");
        }
    (void)hipEventRecord(ev[0], h->stream);
    int rc = qap_orbit_outputs(h, p, y);
    (void)hipEventRecord(ev[1], h->stream);
    const double scale = host_tables(h).scale * gain;
    if (rc == QAP_OK) rc = qap_warm_start_outputs(h, y, scale);
    (void)hipEventRecord(ev[2], h->stream);
    (void)hipStreamSynchronize(h->stream);
    float ms[2] = {0.f, 0.f};
    (void)hipEventElapsedTime(&ms[0], ev[0], ev[1]);
    (void)hipEventElapsedTime(&ms[1], ev[1], ev[2]);
    for (auto &e : ev) (void)hipEventDestroy(e);
    dev_free(h, y);
    if (rc != QAP_OK) return rc;
    if (st) {
        st->orbits = count;
        st->scale = scale;
        st->gain = gain;
        st->ms_mlp = ms[0];
        st->ms_write = ms[1];
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        st->mlp_flops = (double)count * 2.0 * (kFeat * kWidth + kWidth * kWidth + kWidth * kOut);
    }
    return QAP_OK;
}

}  // extern "C"
