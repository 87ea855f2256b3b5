// capi.hip -- host side of the C ABI declared in include/qap_rlt2.h.
//
// One handle owns one device arena (all arrays of one RLT2 state) and one
// stream.  qap_dual_ascent enqueues the kernels of each iteration back to
// back; every kernel first reads the device stop flag, so the host never
// waits inside the loop and the whole loop can be replayed from a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qap_rlt2.h"
#include "kernels.hpp"
#include "lap_block.hpp"

using namespace qap;

namespace {

std::string g_init_error;

size_t round_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct qap_ctx {
    int n = 0, m = 0;
    long long T = 0;
    size_t Vz = 0;
    qap_params prm{};
    // host-derived constants, computed once in FP64
    double kz = 0, okz = 0, phi = 0, ky2 = 0, kx3 = 0, oky = 0, okx = 0, phy = 0, ophy = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // arena
    void *arena = nullptr;
    size_t arena_bytes = 0;
    double *Z = nullptr, *Yc = nullptr, *Py = nullptr;
    double *Xc = nullptr, *Px = nullptr, *alpha = nullptr, *beta = nullptr;
    double *F = nullptr, *D = nullptr, *B = nullptr;
    int *xperm = nullptr, *bestperm = nullptr, *triples = nullptr;
    unsigned long long *bins = nullptr;  // Dijkstra-step counters
    DevScalars *S = nullptr;
    double *trace = nullptr;
    int trace_cap = 0;
    int ntriples = 0;
    int t_host = 0;
    bool integer_data = false;
    int zl = 0, zc = 0;  // Z-LAP mapping
    int zlap_waves = 1;  // waves per Z-LAP block
    bool zl_auto = false;     // mapping left to the autotuner (zlap_lanes = 0)
    bool half = false;        // HALF scheme: only the tiles with i < j are solved
    int sweep_cb = 8;         // cube edge of the ascent sweep (sweep_cube)
    bool sa_on = false;       // Type 4 steps with annealing after each X-LAP
    SaConsts sa{};
    bool zl_tuned = false;    // the autotuner has chosen it
    double zl_tune_us = -1.0; // its time over the tuner's synthetic tiles (< 0: rule-based)
    double offset = 0.0; // constant added to every permutation cost (B&B nodes)
    std::vector<double> hF, hD, hB;
    // host mirror of the arena's small arrays, from F to the step counters
    // (F, D, B, alpha, beta, the two matchings, the triples, the scalar
    // block, the counters: contiguous in the arena), uploaded in one copy at
    // every reset; it lives while the handle does, so no upload waits
    std::vector<char> hsmall;
    bool folded = false;  // a branch-and-bound child: z holds its parent's reduced costs
    std::string err;
    hipGraphExec_t graph = nullptr;  // one full iteration (t >= 1)
    // multiplier tracking (Vz entries like Z, T entries like Yc), or null
    double *Vt = nullptr, *Ut = nullptr;
    // allocator the arena and the bound trace come from (prm.alloc may
    // change later)
    qap_alloc_fn arena_alloc = nullptr;
    qap_free_fn arena_free = nullptr;
    void *arena_ctx = nullptr;
};

namespace {

// Device memory from the handle's arena allocator (hipMalloc without one),
// and back: a caller's allocator without a free function keeps what it gave.
void *arena_mem(qap_ctx *h, size_t bytes)
{
    if (h->arena_alloc) return h->arena_alloc(bytes, h->arena_ctx);
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void arena_mem_free(qap_ctx *h, void *p)
{
    if (!p) return;
    if (!h->arena_alloc)
        (void)hipFree(p);
    else if (h->arena_free)
        h->arena_free(p, h->arena_ctx);
}

int fail(qap_ctx *h, int code, const std::string &msg)
{
    if (h)
        h->err = msg;
    else
        g_init_error = msg;
    return code;
}

#define HIPCHK(h, call)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((h), QAP_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));   \
    } while (0)

bool finite_all(const double *a, int n)
{
    for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

bool integer_all(const double *a, int n)
{
    for (int i = 0; i < n * n; ++i) {
        const double x = a[i];
        if (!(std::fabs(x) < 9.0e15) || x != std::floor(x)) return false;
    }
    return true;
}

struct Sizes {
    size_t z, u, yc, x, nn, trace, tri, total;
};

Sizes sizes_for(int n, int trace_cap)
{
    Sizes s{};
    const long long T = (long long)n * n * (n - 1) * (n - 1);
    const long long m = n - 2;
    const long long ntri = (long long)n * (n - 1) * (n - 2) / 6;
    s.z = round_up(sizeof(double) * (size_t)T * m * m);
    s.u = round_up(sizeof(double) * (size_t)T * m);
    s.yc = round_up(sizeof(double) * (size_t)T);
    s.x = round_up(sizeof(double) * (size_t)n * n);
    s.nn = round_up(sizeof(double) * (size_t)n);
    s.trace = round_up(sizeof(double) * (size_t)trace_cap);
    s.tri = round_up(sizeof(int) * (size_t)std::max<long long>(ntri, 1));
    s.total = s.z + 2 * s.yc + 5 * s.x + 2 * s.nn + 3 * round_up(sizeof(int) * n) + s.tri +
              round_up(sizeof(DevScalars)) + round_up(sizeof(unsigned long long) * kStepBins);
    return s;
}

bool params_ok(const qap_params &p)
{
    auto in01 = [](double x) { return std::isfinite(x) && x >= 0.0 && x <= 1.0; };
    // each member shares among its partners: five under FULL, two upper ones under HALF
    const double partners = p.scheme == QAP_SCHEME_HALF ? 2.0 : 5.0;
    const bool mapping = p.scheme != QAP_SCHEME_HALF || p.zlap_lanes == 0 || p.zlap_lanes == -1;
    const bool variant = (p.two_phase == 0 || (p.two_phase == 1 && p.scheme == QAP_SCHEME_FULL)) &&
                         (p.slow == 0 || (p.slow == 1 && p.scheme == QAP_SCHEME_FULL));
    return (p.scheme == QAP_SCHEME_FULL || p.scheme == QAP_SCHEME_HALF) && mapping && variant && in01(p.kappa_z) &&
           in01(p.kappa_y) && in01(p.kappa_x) && in01(p.phi_z) && in01(p.phi_y) &&
           std::fabs(partners * p.phi_z - 1.0) < 1e-12 && std::isfinite(p.min_gap) && p.min_gap >= 0.0;
}

// Z-LAP lane mapping for size m (lanes per LAP, columns per lane).
void pick_zlap(int m, int req_l, int req_c, int &L, int &C)
{
    if ((req_l == -2 && m <= 32) || req_l == -1) {
        L = req_l;
        C = 1;
        return;
    }
    if (req_l > 0 && req_c > 0 && req_l * req_c >= m) {
        L = req_l;
        C = req_c;
        return;
    }
    // small LAPs: 8/16-lane groups; otherwise the scalar-controlled solver
    // with one 64-lane LAP per wavefront
    C = 1;
    L = m <= 8 ? 8 : m <= 16 ? 16 : -1;
}

template <int L, int C>
hipError_t launch_zlap_t(qap_ctx *h)
{
    const int m = h->m;
    const size_t per = ((size_t)m * m + 2 * m) * sizeof(double);
    const int G = h->zlap_waves * (64 / L);  // whole waves per block
    const long long blocks = (h->T + G - 1) / G;
    hipLaunchKernelGGL((k_zlap<L, C>), dim3((unsigned)blocks), dim3(G * L), G * per, h->stream, h->Z,
                       h->Yc, m, h->T, h->S, h->bins);
    return hipGetLastError();
}

// Tile rows held in registers by the kernels compiled for m = 28 and m = 40
// (k_zlap_s, k_lap_batch_s).  With the whole tile in LDS, LDS limits a CU to
// 24 resident LAPs at m = 28 and 12 at m = 40; with these rows in registers
// the limits are 32 (the wave limit; 54 VGPRs) and 28 (70 VGPRs).
constexpr int kRegRows28 = 16, kRegRows40 = 24;

template <int H>
hipError_t launch_zlap_s(qap_ctx *h)
{
    const int m = h->m;
    const int kr = (H == 1 && m == 28) ? kRegRows28 : (H == 1 && m == 40) ? kRegRows40 : 0;
    // one LAP: the tile's LDS rows, row potentials and one int per column
    // (the solver's proposal and matching slots share it); two LAPs: also v
    // for the epilogue
    const size_t per = H == 1 ? ((size_t)(m - kr) * m + m) * sizeof(double) + ((size_t)m * sizeof(int) + 7) / 8 * 8
                              : ((size_t)m * m + 2 * m) * sizeof(double) * H;
    // HALF: one block per tile with i < j (half of them; H = 1 only)
    const int half = (H == 1 && h->half) ? 1 : 0;
    const long long blocks = half ? h->T / 2 : (h->T + H - 1) / H;
    // the tile sizes of the n = 30 and n = 42 workloads have kernels compiled for them
    if (H == 1 && m == 28)
        hipLaunchKernelGGL((k_zlap_s<1, 28, kRegRows28>), dim3((unsigned)blocks), dim3(64), per, h->stream, h->Z,
                           h->Yc, m, h->T, h->S, h->bins, half);
    else if (H == 1 && m == 40)
        hipLaunchKernelGGL((k_zlap_s<1, 40, kRegRows40>), dim3((unsigned)blocks), dim3(64), per, h->stream, h->Z,
                           h->Yc, m, h->T, h->S, h->bins, half);
    else
        hipLaunchKernelGGL((k_zlap_s<H>), dim3((unsigned)blocks), dim3(64), per, h->stream, h->Z, h->Yc, m,
                           h->T, h->S, h->bins, half);
    return hipGetLastError();
}

hipError_t launch_zlap(qap_ctx *h)
{
    const int L = h->zl, C = h->zc;
    if (L == -2) return launch_zlap_s<2>(h);
    if (L == -1) return launch_zlap_s<1>(h);
    if (L == 8 && C == 1) return launch_zlap_t<8, 1>(h);
    if (L == 16 && C == 1) return launch_zlap_t<16, 1>(h);
    if (L == 32 && C == 1) return launch_zlap_t<32, 1>(h);
    if (L == 64 && C == 1) return launch_zlap_t<64, 1>(h);
    if (L == 8 && C == 2) return launch_zlap_t<8, 2>(h);
    if (L == 16 && C == 2) return launch_zlap_t<16, 2>(h);
    if (L == 32 && C == 2) return launch_zlap_t<32, 2>(h);
    if (L == 8 && C == 4) return launch_zlap_t<8, 4>(h);
    if (L == 16 && C == 4) return launch_zlap_t<16, 4>(h);
    return hipErrorInvalidValue;
}

hipError_t launch_ylap(qap_ctx *h, int equalize)
{
    const int n = h->n, m = n - 1;
    // one Y-LAP per wavefront, scalar-controlled solver
    const size_t per = ((size_t)m * m + m) * sizeof(double) + ((size_t)m * sizeof(int) + 7) / 8 * 8;
    hipLaunchKernelGGL(k_ylap_s, dim3((unsigned)(n * n)), dim3(64), per, h->stream, h->Yc, h->Py, h->Xc, n,
                       equalize, h->ophy, h->phy, h->S, h->bins, h->Ut);
    return hipGetLastError();
}

// Cube edge of the sweep for size n: 10 when its cubes cover the n^3
// locations with fewer slots left over than 8's (n = 9, 10, 17-20, 25-30,
// 49, 50, 57-60), else 8.  A smaller edge (7 at n = 42) wastes no slots there
// but measured slower: shorter runs per cache line and fewer waves per CU.
int sweep_cube(int n)
{
    auto slots = [n](int cb) {
        const long long c = (long long)((n + cb - 1) / cb) * cb;
        return c * c * c;
    };
    return slots(10) < slots(8) ? 10 : 8;
}

template <int CB, bool TRACK, bool HALF, bool POOL, bool SLOW>
hipError_t launch_sweep_cb(qap_ctx *h, const SweepConsts &K, double *Vt)
{
    const unsigned groups8 = (unsigned)((h->ntriples + 7) / 8);
    const int nb = (h->n + CB - 1) / CB;
    const unsigned blocks = groups8 * 8u * (unsigned)(nb * nb * nb);
    hipLaunchKernelGGL((k_sweep<CB, TRACK, HALF, POOL, SLOW>), dim3(blocks), dim3(Cube<CB>::NT), 0, h->stream,
                       h->Z, h->Py, h->Px, h->triples, h->ntriples, h->n, nb, K, h->S, Vt);
    return hipGetLastError();
}

template <bool TRACK, bool HALF, bool POOL, bool SLOW>
hipError_t launch_sweep_k(qap_ctx *h, const SweepConsts &K, double *Vt)
{
    if (h->sweep_cb == 10) return launch_sweep_cb<10, TRACK, HALF, POOL, SLOW>(h, K, Vt);
    return launch_sweep_cb<8, TRACK, HALF, POOL, SLOW>(h, K, Vt);
}

hipError_t launch_sweep(qap_ctx *h)
{
    hipError_t e;
    const SweepConsts K{h->kz, h->okz, h->ky2, h->kx3, h->phi, 1.0 / 3.0};
    const long long work = std::max<long long>(h->T, (long long)h->n * h->n);
    const unsigned sb = (unsigned)std::min<long long>((work + 255) / 256, 65535);
    if (h->prm.slow) {
        if ((e = launch_sweep_k<true, false, false, true>(h, K, h->Vt)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_slow_reset, dim3(sb), dim3(256), 0, h->stream, h->F, h->D, h->B, h->Xc, h->Yc, h->n,
                           h->S);
        return hipGetLastError();
    }
    if (h->half)
        e = launch_sweep_k<false, true, false, false>(h, K, nullptr);
    else if (h->Vt)
        e = launch_sweep_k<true, false, false, false>(h, K, h->Vt);
    else
        e = launch_sweep_k<false, false, false, false>(h, K, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scale_xy, dim3(sb), dim3(256), 0, h->stream, h->Yc, h->Py, h->Xc, h->Px, h->T, h->n * h->n,
                       h->oky, h->okx, h->S);
    return hipGetLastError();
}

// F2 pooling between the two Z-LAP solves (the sweep's transpose, POOL mode).
hipError_t launch_pool(qap_ctx *h)
{
    const SweepConsts K{h->kz, h->okz, h->ky2, h->kx3, h->phi, 1.0 / 3.0};
    if (h->prm.slow)  // S2: the pooling moves the tracked multipliers too
        return launch_sweep_k<true, false, true, false>(h, K, h->Vt);
    return launch_sweep_k<false, false, true, false>(h, K, nullptr);
}

// Z-LAP phase: one solve (F1), or solve, pool, solve (F2 from t = 1 on).
hipError_t launch_zphase(qap_ctx *h, int t)
{
    hipError_t e;
    if ((e = launch_zlap(h)) != hipSuccess) return e;
    if (h->prm.two_phase && t >= 1) {
        if ((e = launch_pool(h)) != hipSuccess) return e;
        if ((e = launch_zlap(h)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_xlap(qap_ctx *h)
{
    hipLaunchKernelGGL(k_xlap, dim3(1), dim3(64), 0, h->stream, h->Xc, h->Px, h->alpha, h->beta, h->F,
                       h->D, h->B, h->xperm, h->bestperm, h->trace, h->n, h->prm.min_gap, h->offset, h->S);
    return hipGetLastError();
}

hipError_t launch_type4(qap_ctx *h)
{
    if (!h->sa_on) return hipSuccess;
    hipLaunchKernelGGL(k_type4, dim3(1), dim3(64), 0, h->stream, h->Px, h->S, h->n, h->sa);
    return hipGetLastError();
}

hipError_t launch_iteration(qap_ctx *h, int t)
{
    hipError_t e;
    if (t >= 1 && (e = launch_sweep(h)) != hipSuccess) return e;
    if ((e = launch_zphase(h, t)) != hipSuccess) return e;
    if ((e = launch_ylap(h, (t >= 1 && !h->prm.slow) ? 1 : 0)) != hipSuccess) return e;  // S1: u stays 0
    if ((e = launch_xlap(h)) != hipSuccess) return e;
    return launch_type4(h);
}

// Same launches with HIP events between the phases (on the handle's stream).
hipError_t launch_iteration_timed(qap_ctx *h, int t, hipEvent_t *ev)
{
    hipError_t e;
    if ((e = hipEventRecord(ev[0], h->stream)) != hipSuccess) return e;
    if (t >= 1 && (e = launch_sweep(h)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev[1], h->stream)) != hipSuccess) return e;
    if ((e = launch_zphase(h, t)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev[2], h->stream)) != hipSuccess) return e;
    if ((e = launch_ylap(h, (t >= 1 && !h->prm.slow) ? 1 : 0)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev[3], h->stream)) != hipSuccess) return e;
    if ((e = launch_xlap(h)) != hipSuccess) return e;
    if ((e = launch_type4(h)) != hipSuccess) return e;
    return hipEventRecord(ev[4], h->stream);
}

int ensure_trace(qap_ctx *h, int need)
{
    if (need <= h->trace_cap) return QAP_OK;
    int cap = std::max(need, 2 * h->trace_cap);
    double *nt = (double *)arena_mem(h, sizeof(double) * cap);
    if (!nt) return fail(h, QAP_ENOMEM, "trace allocation failed");
    if (h->trace) {
        hipError_t e = hipMemcpyAsync(nt, h->trace, sizeof(double) * h->trace_cap, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            arena_mem_free(h, nt);
            return fail(h, QAP_EDEVICE, std::string("trace copy: ") + hipGetErrorString(e));
        }
        arena_mem_free(h, h->trace);
    }
    h->trace = nt;
    h->trace_cap = cap;
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    return QAP_OK;
}

void derive_constants(qap_ctx *h)
{
    const int n = h->n;
    const double c2 = 1.0 / (double)(n - 2);
    const double c3 = 1.0 / ((double)(n - 1) * (double)(n - 2));
    h->kz = h->prm.kappa_z;
    h->okz = 1.0 - h->prm.kappa_z;
    h->oky = 1.0 - h->prm.kappa_y;
    h->okx = 1.0 - h->prm.kappa_x;
    h->ky2 = h->prm.kappa_y * c2;
    h->kx3 = h->prm.kappa_x * c3;
    h->phi = h->prm.phi_z;
    h->phy = h->prm.phi_y;
    h->ophy = 1.0 - h->prm.phi_y;
}

int upload_scalars(qap_ctx *h, double lb, bool sync = true);

// Algorithm 1's initial state.
int upload_initial(qap_ctx *h)
{
    const int n = h->n;
    const int nn = n * n;
    // F, D and B (with the reset scalars) before k_init_xy reads them
    const int rc = upload_scalars(h, 0.0, false);
    if (rc != QAP_OK) return rc;
    const unsigned fb = 4096;
    hipLaunchKernelGGL(k_fill, dim3(fb), dim3(256), 0, h->stream, h->Z, h->Vz, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(fb), dim3(256), 0, h->stream, h->Py, (size_t)h->T, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->stream, h->Px, (size_t)nn, 0.0);
    hipLaunchKernelGGL(k_init_xy, dim3(std::min<long long>((h->T + 255) / 256, 65535)), dim3(256), 0,
                       h->stream, h->F, h->D, h->B, h->Xc, h->Yc, n);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return QAP_OK;
}

// Reset the scalar block (bound lb, no incumbent, t = 0), the step counters
// and the matchings, in one upload of the small arrays (F, D, B and the
// triples come along unchanged).  The source is the handle's host mirror,
// so without sync the upload stays queued on the handle's stream, ahead of
// its next work.  (An earlier reset's upload may still be queued: it writes
// the same region first, so rewriting the mirror is safe.)
int upload_scalars(qap_ctx *h, double lb, bool sync)
{
    DevScalars s{};
    s.lb = lb;
    s.ub = HUGE_VAL;
    s.t = 0;
    s.proven = 0;
    s.integer_data = h->integer_data ? 1 : 0;
    s.stopped = 0;
    s.steps = 0;
    s.best = -HUGE_VAL;
    char *base = h->hsmall.data();
    std::memcpy(base + ((char *)h->S - (char *)h->F), &s, sizeof(s));
    HIPCHK(h, hipMemcpyAsync(h->F, base, h->hsmall.size(), hipMemcpyHostToDevice, h->stream));
    if (sync) HIPCHK(h, hipStreamSynchronize(h->stream));
    h->t_host = 0;
    return QAP_OK;
}

// Dijkstra steps so far: the binned counters of the Z/Y kernels plus the X-LAP's.
int read_steps(qap_ctx *h, const DevScalars &s, unsigned long long &out)
{
    std::vector<unsigned long long> b(kStepBins);
    HIPCHK(h, hipMemcpyAsync(b.data(), h->bins, sizeof(unsigned long long) * kStepBins, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    unsigned long long tot = s.steps;
    for (auto x : b) tot += x;
    out = tot;
    return QAP_OK;
}

uint64_t fnv1a(uint64_t hsh, const void *data, size_t bytes)
{
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < bytes; ++i) {
        hsh ^= p[i];
        hsh *= 1099511628211ull;
    }
    return hsh;
}

// Allocate and (optionally) initialise a context of size n.  stream: a
// caller stream to share (not owned) or nullptr for a new one.  With init the
// state is Algorithm 1's initial one; otherwise the caller fills Xc, Yc and Z
// (the child fold) and resets the scalars (upload_scalars).
int create_ctx(int n, const double *F, const double *D, const double *B, const qap_params &prm, double offset,
               hipStream_t stream, bool init, qap_ctx **out)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, QAP_EDEVICE, "no HIP device");
    if (prm.device < 0 || prm.device >= ndev) return fail(nullptr, QAP_EINVAL, "bad device ordinal");
    if (hipSetDevice(prm.device) != hipSuccess) return fail(nullptr, QAP_EDEVICE, "hipSetDevice failed");

    const int trace_cap = 1024;
    Sizes sz = sizes_for(n, trace_cap);
    // (a caller's allocator may serve the arena from memory it already holds)
    size_t freeb = 0, totalb = 0;
    if (!prm.alloc && hipMemGetInfo(&freeb, &totalb) != hipSuccess)
        return fail(nullptr, QAP_EDEVICE, "hipMemGetInfo failed");
    if (!prm.alloc && sz.total + sz.trace > freeb) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "arena of %zu bytes exceeds free device memory (%zu)", sz.total + sz.trace,
                      freeb);
        return fail(nullptr, QAP_ENOMEM, buf);
    }

    qap_ctx *h = new qap_ctx();
    h->n = n;
    h->m = n - 2;
    h->T = (long long)n * n * (n - 1) * (n - 1);
    h->Vz = (size_t)h->T * h->m * h->m;
    h->prm = prm;
    h->offset = offset;
    h->hF.assign(F, F + n * n);
    h->hD.assign(D, D + n * n);
    h->hB.assign(n * n, 0.0);
    if (B) h->hB.assign(B, B + n * n);
    h->integer_data = integer_all(F, n) && integer_all(D, n) && integer_all(h->hB.data(), n) &&
                      std::fabs(offset) < 9.0e15 && offset == std::floor(offset);
    derive_constants(h);
    h->sweep_cb = sweep_cube(n);
    h->half = prm.scheme == QAP_SCHEME_HALF;
    // HALF solves the upper tiles with the scalar solver (one LAP per wave)
    pick_zlap(h->m, h->half ? -1 : prm.zlap_lanes, prm.zlap_cols, h->zl, h->zc);
    h->zl_auto = !h->half && prm.zlap_lanes == 0;

    auto cleanup = [&](int code) {
        const std::string e = h->err;
        qap_destroy(h);
        if (!e.empty()) g_init_error = e;
        return code;
    };
    if (stream) {
        h->stream = stream;
        h->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            delete h;
            return fail(nullptr, QAP_EDEVICE, "stream creation failed");
        }
        h->own_stream = true;
    }
    h->arena_bytes = sz.total;
    void *mem = nullptr;
    if (prm.alloc)
        mem = prm.alloc(h->arena_bytes, prm.alloc_ctx);
    else if (hipMalloc(&mem, h->arena_bytes) != hipSuccess)
        mem = nullptr;
    if (!mem) {
        g_init_error = "device arena allocation failed";
        return cleanup(QAP_ENOMEM);
    }
    h->arena = mem;
    h->arena_alloc = prm.alloc;
    h->arena_free = prm.free_fn;
    h->arena_ctx = prm.alloc_ctx;
    char *c = (char *)mem;
    auto take = [&](size_t bytes) {
        char *r = c;
        c += bytes;
        return (void *)r;
    };
    h->Z = (double *)take(sz.z);
    h->Yc = (double *)take(sz.yc);
    h->Py = (double *)take(sz.yc);
    h->Xc = (double *)take(sz.x);
    h->Px = (double *)take(sz.x);
    h->F = (double *)take(sz.x);
    h->D = (double *)take(sz.x);
    h->B = (double *)take(sz.x);
    h->alpha = (double *)take(sz.nn);
    h->beta = (double *)take(sz.nn);
    h->xperm = (int *)take(round_up(sizeof(int) * n));
    h->bestperm = (int *)take(round_up(sizeof(int) * n));
    take(round_up(sizeof(int) * n));
    h->triples = (int *)take(sz.tri);
    h->S = (DevScalars *)take(round_up(sizeof(DevScalars)));
    h->bins = (unsigned long long *)take(round_up(sizeof(unsigned long long) * kStepBins));
    h->trace = (double *)arena_mem(h, sizeof(double) * trace_cap);
    if (!h->trace) {
        g_init_error = "trace allocation failed";
        return cleanup(QAP_ENOMEM);
    }
    h->trace_cap = trace_cap;

    // the host mirror of the small arrays: F, D, B, zero duals, identity
    // matchings, the facility triples i<j<k (packed 8 bits each), a scalar
    // block (set by each reset), zero step counters
    h->hsmall.assign((char *)(h->bins + kStepBins) - (char *)h->F, 0);
    {
        char *base = h->hsmall.data();
        auto at = [&](const void *dev) { return base + ((const char *)dev - (const char *)h->F); };
        const size_t nnb = sizeof(double) * (size_t)n * n;
        std::memcpy(at(h->F), h->hF.data(), nnb);
        std::memcpy(at(h->D), h->hD.data(), nnb);
        std::memcpy(at(h->B), h->hB.data(), nnb);
        int *xp = (int *)at(h->xperm), *bp = (int *)at(h->bestperm);
        for (int i = 0; i < n; ++i) xp[i] = bp[i] = i;
        int *tp = (int *)at(h->triples);
        int nt = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                for (int k = j + 1; k < n; ++k) tp[nt++] = i | (j << 8) | (k << 16);
        h->ntriples = nt;
    }
    // without init the caller fills the arrays and resets the scalars (the
    // reset uploads the mirror)
    if (init) {
        const int rc = upload_initial(h);
        if (rc != QAP_OK) return cleanup(rc);
    }
    *out = h;
    return QAP_OK;
}

}  // namespace

#include "tune_host.hpp"

extern "C" {

const char *qap_version(void) { return "qap-rlt2-mi355x 0.1 (gfx950, F1, F2 and S1; FULL and HALF; Type 4)"; }

int qap_set_annealing(qap_handle h, const qap_sa_params *p)
{
    if (!h) return QAP_EINVAL;
    const bool on = p && p->t0 > 0.0;
    if (on) {
        if (!std::isfinite(p->t0) || !(p->kappa_max >= 0.0 && p->kappa_max <= 1.0) ||
            !(p->cool > 0.0 && p->cool <= 1.0) || p->period < 1)
            return fail(h, QAP_EINVAL, "annealing needs t0 > 0 finite, kappa_max in [0,1], cool in (0,1], period >= 1");
        if (h->Vt || h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "annealing does not combine with multiplier tracking or S1");
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->sa_on = on;
    if (on) h->sa = SaConsts{p->t0, p->kappa_max, p->cool, p->seed, p->period};
    if (h->graph) {  // the next replay captures the iteration with (or without) the step
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    return QAP_OK;
}

int qap_zlap_mapping(qap_handle h, int *lanes, int *cols, double *tuned_us)
{
    if (!h) return QAP_EINVAL;
    if (lanes) *lanes = h->zl;
    if (cols) *cols = h->zc;
    if (tuned_us) *tuned_us = h->zl_tuned ? h->zl_tune_us : -1.0;
    return QAP_OK;
}

int qap_default_params(qap_params *p)
{
    if (!p) return QAP_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->kappa_z = 5.0 / 6.0;
    p->kappa_y = 1.0;
    p->kappa_x = 1.0;
    p->phi_z = 1.0 / 5.0;
    p->phi_y = 0.5;
    p->min_gap = 0.0;
    return QAP_OK;
}

size_t qap_workspace_bytes(int n, const qap_params *p)
{
    (void)p;
    if (n < 3 || n > 64) return 0;
    return sizes_for(n, 1024).total + round_up(sizeof(double) * 1024);
}

int qap_rlt2_init(const double *F, const double *D, const double *B, int n, const qap_params *p,
                  qap_handle *out)
{
    if (!out) return fail(nullptr, QAP_EINVAL, "out is NULL");
    if (n < 3 || n > 64) return fail(nullptr, QAP_EUNSUPPORTED, "n must be in 3..64");
    if (!F || !D) return fail(nullptr, QAP_EINVAL, "F and D are required");
    if (!finite_all(F, n) || !finite_all(D, n) || (B && !finite_all(B, n)))
        return fail(nullptr, QAP_EINVAL, "non-finite input entry");
    qap_params prm;
    if (p)
        prm = *p;
    else
        qap_default_params(&prm);
    if (!params_ok(prm))
        return fail(nullptr, QAP_EINVAL,
                    "kappa/phi outside [0,1], phi_z not 1/5 (FULL) or 1/2 (HALF), or bad scheme/mapping/variant");
    return create_ctx(n, F, D, B, prm, 0.0, nullptr, true, out);
}

int qap_destroy(qap_handle h)
{
    if (!h) return QAP_EINVAL;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->arena) {
        if (h->arena_alloc && h->arena_free)
            h->arena_free(h->arena, h->arena_ctx);
        else if (!h->arena_alloc)
            (void)hipFree(h->arena);
    }
    arena_mem_free(h, h->trace);
    for (double *a : {h->Vt, h->Ut}) {
        if (!a) continue;
        if (h->prm.alloc && h->prm.free_fn)
            h->prm.free_fn(a, h->prm.alloc_ctx);
        else if (!h->prm.alloc)
            (void)hipFree(a);
    }
    if (h->stream && h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return QAP_OK;
}

int qap_set_stream(qap_handle h, void *hip_stream)
{
    if (!h) return QAP_EINVAL;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    h->stream = (hipStream_t)hip_stream;
    h->own_stream = false;
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    return QAP_OK;
}

int qap_dual_ascent(qap_handle h, int iters, double *lb_out, double *alpha_out, double *beta_out,
                    qap_da_stats *st)
{
    if (!h) return QAP_EINVAL;
    if (iters < 0) return fail(h, QAP_EINVAL, "iters < 0");
    HIPCHK(h, hipSetDevice(h->prm.device));
    if (h->prm.slow && !h->Vt && iters > 0) {
        // S1 keeps its z multipliers in the tracking array from the start
        const int rc = qap_track(h, 1);
        if (rc != QAP_OK) return rc;
    }
    if (h->zl_auto && !h->zl_tuned && iters > 0) {
        // pick the Z-LAP mapping by measurement before anything is captured
        HIPCHK(h, hipStreamSynchronize(h->stream));
        tune_handle_zlap(h);
        if (h->graph) {
            (void)hipGraphExecDestroy(h->graph);
            h->graph = nullptr;
        }
    }
    auto t0 = std::chrono::steady_clock::now();
    DevScalars before{};
    HIPCHK(h, hipMemcpyAsync(&before, h->S, sizeof(before), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->t_host = before.t;
    unsigned long long steps_before = 0, steps_after = 0;
    if (st) {
        int rs = read_steps(h, before, steps_before);
        if (rs != QAP_OK) return rs;
    }
    int rc = ensure_trace(h, h->t_host + iters + 1);
    if (rc != QAP_OK) return rc;
    std::vector<hipEvent_t> evs;
    if (h->prm.timing) {
        evs.resize((size_t)5 * iters);
        for (auto &e : evs) HIPCHK(h, hipEventCreate(&e));
    }
    for (int it = 0; it < iters; ++it) {
        const int t = h->t_host + it;
        if (h->prm.timing) {
            hipError_t e = launch_iteration_timed(h, t, &evs[(size_t)5 * it]);
            if (e != hipSuccess) return fail(h, QAP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
        } else if (t >= 1 && h->stream != nullptr) {
            // graph replay (the legacy null stream cannot be captured: there
            // the iterations are launched one kernel at a time below)
            if (!h->graph) {
                hipGraph_t g = nullptr;
                HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
                hipError_t le = launch_iteration(h, 1);
                hipError_t ce = hipStreamEndCapture(h->stream, &g);
                if (le != hipSuccess) return fail(h, QAP_EDEVICE, std::string("launch: ") + hipGetErrorString(le));
                if (ce != hipSuccess) return fail(h, QAP_EDEVICE, std::string("capture: ") + hipGetErrorString(ce));
                hipError_t ie = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return fail(h, QAP_EDEVICE, std::string("instantiate: ") + hipGetErrorString(ie));
            }
            HIPCHK(h, hipGraphLaunch(h->graph, h->stream));
        } else {
            hipError_t e = launch_iteration(h, t);
            if (e != hipSuccess) return fail(h, QAP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
        }
    }
    DevScalars after{};
    HIPCHK(h, hipMemcpyAsync(&after, h->S, sizeof(after), hipMemcpyDeviceToHost, h->stream));
    std::vector<double> a(h->n), b(h->n);
    HIPCHK(h, hipMemcpyAsync(a.data(), h->alpha, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(b.data(), h->beta, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    auto t1 = std::chrono::steady_clock::now();
    double ph[4] = {0, 0, 0, 0};
    for (int it = 0; it < (h->prm.timing ? iters : 0); ++it) {
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            HIPCHK(h, hipEventElapsedTime(&ms, evs[(size_t)5 * it + k], evs[(size_t)5 * it + k + 1]));
            ph[k] += ms;
        }
    }
    for (auto &e : evs) (void)hipEventDestroy(e);
    h->t_host = after.t;
    if (lb_out) *lb_out = after.lb;
    if (alpha_out) std::memcpy(alpha_out, a.data(), sizeof(double) * h->n);
    if (beta_out) std::memcpy(beta_out, b.data(), sizeof(double) * h->n);
    if (st) {
        st->iterations_done = after.t - before.t;
        st->t = after.t;
        st->lb = after.lb;
        st->best_lb = after.best;
        st->sa_steps = after.sa_steps;
        st->ub = after.ub;
        const double bl = std::max(after.lb, after.best);
        st->gap = (after.ub < HUGE_VAL && after.ub != 0.0) ? (after.ub - bl) / std::fabs(after.ub) : HUGE_VAL;
        st->proven = after.proven;
        const long long zlaps = h->half ? h->T / 2 : h->T;  // HALF: tiles with i < j
        st->laps = (long long)st->iterations_done * (zlaps + (long long)h->n * h->n + 1);
        if (h->prm.two_phase)  // F2 solves the Z-LAPs twice at t >= 1
            st->laps += (long long)std::max(0, after.t - std::max(before.t, 1)) * zlaps;
        int rs = read_steps(h, after, steps_after);
        if (rs != QAP_OK) return rs;
        st->dijkstra_steps = (long long)(steps_after - steps_before);
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        st->ms_sweep = ph[0];
        st->ms_zlap = ph[1];
        st->ms_ylap = ph[2];
        st->ms_xlap = ph[3];
    }
    return QAP_OK;
}

int qap_get_trace(qap_handle h, double *lb, int cap, int *len)
{
    if (!h) return QAP_EINVAL;
    DevScalars s{};
    HIPCHK(h, hipMemcpyAsync(&s, h->S, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (len) *len = s.t;
    const int k = std::min(cap, s.t);
    if (lb && k > 0) {
        HIPCHK(h, hipMemcpyAsync(lb, h->trace, sizeof(double) * k, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return QAP_OK;
}

int qap_get_assignment(qap_handle h, int32_t *xperm, int32_t *best_perm)
{
    if (!h) return QAP_EINVAL;
    if (xperm) HIPCHK(h, hipMemcpyAsync(xperm, h->xperm, sizeof(int) * h->n, hipMemcpyDeviceToHost, h->stream));
    if (best_perm)
        HIPCHK(h, hipMemcpyAsync(best_perm, h->bestperm, sizeof(int) * h->n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return QAP_OK;
}

int qap_export_state(qap_handle h, qap_state_header *hdr, double *x, double *y, double *z)
{
    if (!h) return QAP_EINVAL;
    DevScalars s{};
    HIPCHK(h, hipMemcpyAsync(&s, h->S, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int n = h->n, m = h->m;
    const size_t nn = (size_t)n * n;
    std::vector<double> hx(nn), hy((size_t)h->T), hz;
    const bool post = s.t > 0;
    HIPCHK(h, hipMemcpy(hx.data(), post ? h->Px : h->Xc, sizeof(double) * nn, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(hy.data(), post ? h->Py : h->Yc, sizeof(double) * h->T, hipMemcpyDeviceToHost));
    uint64_t cs = 1469598103934665603ull;
    if (z || hdr) {
        hz.resize(h->Vz);
        HIPCHK(h, hipMemcpy(hz.data(), h->Z, sizeof(double) * h->Vz, hipMemcpyDeviceToHost));
    }
    if (hdr) {
        hdr->n = n;
        hdr->t = s.t;
        hdr->lb = s.lb;
        hdr->ub = s.ub;
        cs = fnv1a(cs, &hdr->n, sizeof(int));
        cs = fnv1a(cs, &hdr->t, sizeof(int));
        cs = fnv1a(cs, &hdr->lb, sizeof(double));
        cs = fnv1a(cs, &hdr->ub, sizeof(double));
        cs = fnv1a(cs, hx.data(), sizeof(double) * hx.size());
        cs = fnv1a(cs, hy.data(), sizeof(double) * hy.size());
        cs = fnv1a(cs, hz.data(), sizeof(double) * hz.size());
        hdr->checksum = cs;
    }
    if (x) std::memcpy(x, hx.data(), sizeof(double) * nn);
    if (y) std::memcpy(y, hy.data(), sizeof(double) * hy.size());
    if (z) std::memcpy(z, hz.data(), sizeof(double) * hz.size());
    return QAP_OK;
}

int qap_export_z_tiles(qap_handle h, const int64_t *tiles, int count, double *out)
{
    if (!h || count < 0 || (count > 0 && (!tiles || !out))) return QAP_EINVAL;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int m = h->m;
    const size_t mm = (size_t)m * m;
    for (int a = 0; a < count; ++a) {
        const int64_t t = tiles[a];
        if (t < 0 || t >= h->T) return fail(h, QAP_EINVAL, "tile index out of range");
        double *dst = out + (size_t)a * mm;
        HIPCHK(h, hipMemcpy(dst, h->Z + (size_t)t * mm, sizeof(double) * mm, hipMemcpyDeviceToHost));
    }
    return QAP_OK;
}

int qap_import_state(qap_handle h, const qap_state_header *hdr, const double *x, const double *y,
                     const double *z)
{
    if (!h || !hdr || !x || !y || !z) return QAP_EINVAL;
    if (hdr->n != h->n || hdr->t < 0) return fail(h, QAP_ESTATE, "state header does not match the handle");
    const size_t nn = (size_t)h->n * h->n;
    uint64_t cs = 1469598103934665603ull;
    cs = fnv1a(cs, &hdr->n, sizeof(int));
    cs = fnv1a(cs, &hdr->t, sizeof(int));
    cs = fnv1a(cs, &hdr->lb, sizeof(double));
    cs = fnv1a(cs, &hdr->ub, sizeof(double));
    cs = fnv1a(cs, x, sizeof(double) * nn);
    cs = fnv1a(cs, y, sizeof(double) * h->T);
    cs = fnv1a(cs, z, sizeof(double) * h->Vz);
    if (cs != hdr->checksum) return fail(h, QAP_ESTATE, "state checksum mismatch");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "an S1 state lives in its multipliers, not in the costs");
    if (h->half) {
        // tiles (i,p,j',q') with j < i, i.e. j' < i, must hold zeros
        const int n = h->n;
        const size_t mm = (size_t)h->m * h->m;
        for (long long t = 0; t < h->T; ++t) {
            const long long ip = t / ((long long)(n - 1) * (n - 1));
            const int jp = (int)((t / (n - 1)) % (n - 1));
            if (jp >= ip / n) continue;
            for (size_t a = 0; a < mm; ++a)
                if (z[t * mm + a] != 0.0) return fail(h, QAP_EINVAL, "HALF state with a nonzero lower z entry");
        }
    }
    const bool post = hdr->t > 0;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(post ? h->Px : h->Xc, x, sizeof(double) * nn, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(post ? h->Py : h->Yc, y, sizeof(double) * h->T, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->Z, z, sizeof(double) * h->Vz, hipMemcpyHostToDevice));
    DevScalars s{};
    HIPCHK(h, hipMemcpyAsync(&s, h->S, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    s.lb = hdr->lb;
    s.ub = hdr->ub;
    s.t = hdr->t;
    s.proven = 0;
    s.stopped = 0;
    s.best = hdr->t > 0 ? hdr->lb : -HUGE_VAL;
    HIPCHK(h, hipMemcpyAsync(h->S, &s, sizeof(s), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->t_host = hdr->t;
    return QAP_OK;
}

int qap_lap_batch(const double *cost, int count, int m, double *u, double *v, double *theta,
                  int32_t *row_of_col, int lanes, int cols, void *stream)
{
    if (m < 1 || m > kBlockLap * 4 || count < 0) return fail(nullptr, QAP_EINVAL, "m must be 1..1024, count >= 0");
    if (count == 0) return QAP_OK;
    if (!cost || !u || !v || !theta || !row_of_col) return fail(nullptr, QAP_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    if (m > 64) {
        // larger than a wavefront: one LAP per block of kBlockLap threads,
        // the matrix read from global memory
        const int Cb = (m + kBlockLap - 1) / kBlockLap;
        const size_t lb = block_lap_lds_bytes(m);
#define QAP_LBB(CC)                                                                                             \
    if (Cb == CC)                                                                                               \
        hipLaunchKernelGGL((k_lap_block<CC>), dim3((unsigned)count), dim3(kBlockLap), lb, s, cost, count, m, u, v, \
                           theta, (int *)row_of_col);
        QAP_LBB(1) QAP_LBB(2) QAP_LBB(3) QAP_LBB(4)
#undef QAP_LBB
        HIPCHK(nullptr, hipGetLastError());
        return QAP_OK;
    }
    int L, C;
    pick_zlap(m, lanes, cols, L, C);
    const size_t per = ((size_t)m * m + 2 * m) * sizeof(double);
    int G = 256 / L;
    while (G > 1 && (size_t)G * per > 65536) --G;
    const unsigned blocks = (unsigned)((count + G - 1) / G);
#define QAP_LB(LL, CC)                                                                                   \
    if (L == LL && C == CC) {                                                                            \
        hipLaunchKernelGGL((k_lap_batch<LL, CC>), dim3(blocks), dim3(G * LL), G * per, s, cost, count, m, \
                           u, v, theta, (int *)row_of_col);                                              \
    } else
    QAP_LB(8, 1) QAP_LB(16, 1) QAP_LB(32, 1) QAP_LB(64, 1) QAP_LB(8, 2) QAP_LB(16, 2) QAP_LB(32, 2)
    QAP_LB(8, 4) QAP_LB(16, 4)
    if (L == -2 || L == -1) {
        const int H = -L;
        const size_t pers = ((size_t)m * m + 2 * m) * sizeof(double) * H;
        const unsigned bs = (unsigned)((count + H - 1) / H);
        if (H == 2)
            hipLaunchKernelGGL((k_lap_batch_s<2>), dim3(bs), dim3(64), pers, s, cost, count, m, u, v, theta,
                               (int *)row_of_col);
        else if (m == 28)  // the tile sizes with kernels compiled for them (k_zlap_s)
            hipLaunchKernelGGL((k_lap_batch_s<1, 28, kRegRows28>), dim3(bs), dim3(64), pers, s, cost, count, m, u, v,
                               theta, (int *)row_of_col);
        else if (m == 40)
            hipLaunchKernelGGL((k_lap_batch_s<1, 40, kRegRows40>), dim3(bs), dim3(64), pers, s, cost, count, m, u, v,
                               theta, (int *)row_of_col);
        else
            hipLaunchKernelGGL((k_lap_batch_s<1>), dim3(bs), dim3(64), pers, s, cost, count, m, u, v, theta,
                               (int *)row_of_col);
    } else {
        return fail(nullptr, QAP_EINVAL, "unsupported lanes/cols mapping");
    }
#undef QAP_LB
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, QAP_EDEVICE, hipGetErrorString(e));
    return QAP_OK;
}

const char *qap_last_error(qap_handle h)
{
    if (!h) return g_init_error.c_str();
    return h->err.c_str();
}

}  // extern "C"

#include "bnb_host.hpp"
#include "learn_host.hpp"
