// bnb_host.hpp -- host side of the child fold, the batched dual ascent and
// the branch-and-bound of Section 4 (included at the end of capi.hip: one
// translation unit with the context helpers).
#pragma once
#include <algorithm>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "batch.hpp"

namespace {

// Device memory of a search's node handles (arenas and bound traces).  A
// hipFree costs a few hundred microseconds, so blocks come from slabs of up
// to 1 GiB that hold several blocks of one size (all nodes of one size need
// the same bytes); a block freed by a finished node goes back to its size's
// free list for a later node, and the slabs are freed when the search ends.
struct NodeArenaPool {
    static constexpr size_t kSlab = (size_t)1 << 30;
    static constexpr size_t kMaxPerSlab = 64;
    std::unordered_map<size_t, std::vector<void *>> free_blocks;  // by block size
    std::unordered_map<void *, size_t> size_of;                  // block -> its size
    std::vector<void *> slabs;

    static void *alloc(size_t bytes, void *ctx)
    {
        NodeArenaPool &P = *(NodeArenaPool *)ctx;
        const size_t bsz = round_up(bytes);
        std::vector<void *> &fl = P.free_blocks[bsz];
        if (fl.empty()) {
            const size_t k = std::max<size_t>(1, std::min(kMaxPerSlab, kSlab / bsz));
            char *slab = nullptr;
            if (hipMalloc((void **)&slab, k * bsz) != hipSuccess) return nullptr;
            P.slabs.push_back(slab);
            for (size_t i = k; i-- > 0;) {
                fl.push_back(slab + i * bsz);
                P.size_of[slab + i * bsz] = bsz;
            }
        }
        void *p = fl.back();
        fl.pop_back();
        return p;
    }
    static void release(void *p, void *ctx)
    {
        NodeArenaPool &P = *(NodeArenaPool *)ctx;
        const auto it = P.size_of.find(p);
        if (it != P.size_of.end()) P.free_blocks[it->second].push_back(p);
    }
    NodeArenaPool() = default;
    NodeArenaPool(const NodeArenaPool &) = delete;
    NodeArenaPool &operator=(const NodeArenaPool &) = delete;
    ~NodeArenaPool()
    {
        for (void *s : slabs) (void)hipFree(s);
    }
};

bool fathomed_host(double lb, double ub, bool integer_data)
{
    if (!(ub < HUGE_VAL)) return false;
    const double tol = 1e-9 * std::fmax(1.0, std::fabs(ub));
    if (integer_data) return std::ceil(lb - tol) >= ub;
    return lb >= ub - tol;
}

// Exact QAP cost of a full permutation (int64 when every input is integer).
double full_cost(const qap_ctx *root, const std::vector<int> &perm)
{
    const int n = root->n;
    const double *F = root->hF.data(), *D = root->hD.data(), *B = root->hB.data();
    if (root->integer_data) {
        long long c = 0;
        for (int i = 0; i < n; ++i) {
            c += (long long)B[i * n + perm[i]];
            for (int j = 0; j < n; ++j) c += (long long)F[i * n + j] * (long long)D[perm[i] * n + perm[j]];
        }
        return (double)c;
    }
    long double c = 0.0L;
    for (int i = 0; i < n; ++i) {
        c += B[i * n + perm[i]];
        for (int j = 0; j < n; ++j) c += (long double)F[i * n + j] * D[perm[i] * n + perm[j]];
    }
    return (double)c;
}

// Rule 3 (Section 4): lowest total interaction first, then the lowest summed
// interaction with the facilities already placed; ties to the lowest index.
std::vector<int> rule3_order(int n, const double *F)
{
    std::vector<int> order, placed(n, 0);
    for (int t = 0; t < n; ++t) {
        int best = -1;
        double bv = HUGE_VAL;
        for (int i = 0; i < n; ++i) {
            if (placed[i]) continue;
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                if (t == 0) {
                    if (j != i) s += F[i * n + j] + F[j * n + i];
                } else if (placed[j]) {
                    s += F[i * n + j] + F[j * n + i];
                }
            }
            if (s < bv) {
                bv = s;
                best = i;
            }
        }
        order.push_back(best);
        placed[best] = 1;
    }
    return order;
}

// Location automorphisms for the symmetry elimination of Section 4 (grid
// instances): permutations sigma of the locations with D[sigma p][sigma q] =
// D[p][q] for all p, q and B[i][sigma p] = B[i][p] for all i, p, so that
// placing every facility at sigma of its location keeps the cost.  Depth-
// first over p = 0, 1, ... with candidates of equal sorted row, sorted column
// and B column; each permutation found satisfies the equalities exactly.
// Stops after `cap` permutations or a step budget, so on a highly symmetric
// D it may return a subset (the identity first): any subset of exact
// automorphisms keeps the elimination exact.
std::vector<std::vector<int>> location_automorphisms(int n, const double *D, const double *B, int cap)
{
    std::vector<std::vector<double>> sig(n);
    for (int p = 0; p < n; ++p) {
        std::vector<double> row(D + (size_t)p * n, D + (size_t)p * n + n), col(n), bc(n);
        for (int q = 0; q < n; ++q) col[q] = D[(size_t)q * n + p];
        for (int i = 0; i < n; ++i) bc[i] = B ? B[(size_t)i * n + p] : 0.0;
        std::sort(row.begin(), row.end());
        std::sort(col.begin(), col.end());
        sig[p].push_back(D[(size_t)p * n + p]);
        sig[p].insert(sig[p].end(), row.begin(), row.end());
        sig[p].insert(sig[p].end(), col.begin(), col.end());
        sig[p].insert(sig[p].end(), bc.begin(), bc.end());  // B column exactly, not sorted
    }
    std::vector<std::vector<int>> cand(n);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (sig[q] == sig[p]) cand[p].push_back(q);
    std::vector<std::vector<int>> out;
    std::vector<int> sigma(n, -1), used(n, 0);
    long long steps = 0;
    const long long budget = 4000000;
    // iterative depth-first search: pos[k] = next candidate index for p = k
    std::vector<int> pos(n + 1, 0);
    int k = 0;
    while (k >= 0 && (int)out.size() < cap && steps < budget) {
        if (k == n) {
            out.push_back(sigma);
            --k;
            used[sigma[k]] = 0;
            sigma[k] = -1;
            continue;
        }
        bool placed = false;
        while (pos[k] < (int)cand[k].size()) {
            const int q = cand[k][pos[k]++];
            ++steps;
            if (used[q]) continue;
            bool ok = D[(size_t)q * n + q] == D[(size_t)k * n + k];
            for (int t = 0; ok && t < k; ++t)
                ok = D[(size_t)q * n + sigma[t]] == D[(size_t)k * n + t] &&
                     D[(size_t)sigma[t] * n + q] == D[(size_t)t * n + k];
            if (!ok) continue;
            sigma[k] = q;
            used[q] = 1;
            placed = true;
            break;
        }
        if (placed) {
            ++k;
            if (k < n) pos[k] = 0;
        } else {
            pos[k] = 0;
            --k;
            if (k >= 0) {
                used[sigma[k]] = 0;
                sigma[k] = -1;
            }
        }
    }
    return out;
}

// Workspace of qap_batch_dual_ascent_static: the batch's node table,
// prefix tables and stop counter.  Each GPU holds its own copy of the array
// until the process ends; in host code its name is only a stand-in, so the
// device address is taken once per device (hipGetSymbolAddress, with that
// device current) and used everywhere host code needs the memory.
static __device__ __align__(256) char scratch[QAP_BATCH_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on h's device (set-up on the first call
// on that device).
int static_workspace(qap_ctx *h, char **ws)
{
    const int dev = h->prm.device;
    if (dev < 0 || dev >= kMaxDevices) return fail(h, QAP_EUNSUPPORTED, "device ordinal beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        HIPCHK(h, hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(h, QAP_EDEVICE, std::string("static workspace: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)p;
    }
    *ws = g_scratch_ptr[dev];
    return QAP_OK;
}

}  // namespace

extern "C" {

int qap_location_automorphisms(int n, const double *D, const double *B, int cap, int32_t *out, int *count)
{
    if (n < 1 || n > 64 || !D || cap < 1 || !out || !count) return fail(nullptr, QAP_EINVAL, "bad arguments");
    const auto g = location_automorphisms(n, D, B, cap);
    for (size_t a = 0; a < g.size(); ++a)
        for (int p = 0; p < n; ++p) out[a * n + p] = g[a][p];
    *count = (int)g.size();
    return QAP_OK;
}

}  // extern "C"

namespace {

// The child fold once the parent's bound plus pi_x[l][s] (the child's
// starting bound) is known on the host; arguments already checked.  Every
// step is queued on the parent's stream, which the child shares.
int fold_core(qap_ctx *h, int l, int s, double child_lb, qap_ctx **child)
{
    const int n = h->n, n1 = n - 1;
    // the child's own QAP: F, D restricted, fixed pair folded into B, constant
    const double *F = h->hF.data(), *D = h->hD.data(), *B = h->hB.data();
    std::vector<double> Fc((size_t)n1 * n1), Dc((size_t)n1 * n1), Bc((size_t)n1 * n1);
    for (int a1 = 0; a1 < n1; ++a1)
        for (int a2 = 0; a2 < n1; ++a2) {
            const int i = a1 + (a1 >= l), j = a2 + (a2 >= l);
            const int p = a1 + (a1 >= s), q = a2 + (a2 >= s);
            Fc[(size_t)a1 * n1 + a2] = F[i * n + j];
            Dc[(size_t)a1 * n1 + a2] = D[p * n + q];
            Bc[(size_t)a1 * n1 + a2] = (B[i * n + q] + F[i * n + l] * D[q * n + s]) + F[l * n + i] * D[s * n + q];
        }
    const double off = h->offset + (B[l * n + s] + F[l * n + l] * D[s * n + s]);
    qap_ctx *c = nullptr;
    int rc = create_ctx(n1, Fc.data(), Dc.data(), Bc.data(), h->prm, off, h->stream, false, &c);
    if (rc != QAP_OK) {
        h->err = g_init_error;
        return rc;
    }
    const long long T1 = c->T;
    const unsigned gxy = (unsigned)std::min<long long>((T1 + (long long)n1 * n1 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fold_xy, dim3(gxy), dim3(256), 0, h->stream, h->Px, h->Py, h->Z, n, l, s, c->Xc, c->Yc);
    const unsigned gz = (unsigned)std::min<long long>(((long long)c->Vz + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fold_z, dim3(gz), dim3(256), 0, h->stream, h->Z, n, l, s, c->Z);
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(256), 0, h->stream, c->Py, (size_t)T1, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->stream, c->Px, (size_t)n1 * n1, 0.0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qap_destroy(c);
        return fail(h, QAP_EDEVICE, std::string("fold: ") + hipGetErrorString(e));
    }
    rc = upload_scalars(c, child_lb, false);
    if (rc != QAP_OK) {
        h->err = c->err;
        qap_destroy(c);
        return rc;
    }
    c->folded = true;
    *child = c;
    return QAP_OK;
}

}  // namespace

extern "C" {

int qap_fold_child(qap_handle h, int l, int s, qap_handle *child)
{
    if (!h || !child) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound children are FULL-scheme only");
    if (h->prm.two_phase) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound children are F1 only");
    if (h->sa_on) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound children run without annealing");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound children are F1 only");
    const int n = h->n;
    if (n - 1 < 3) return fail(h, QAP_EUNSUPPORTED, "a child needs n >= 4");
    if (l < 0 || l >= n || s < 0 || s >= n) return fail(h, QAP_EINVAL, "facility/location out of range");
    DevScalars ps{};
    HIPCHK(h, hipMemcpyAsync(&ps, h->S, sizeof(ps), hipMemcpyDeviceToHost, h->stream));
    double px = 0.0;
    HIPCHK(h, hipMemcpyAsync(&px, h->Px + (size_t)l * n + s, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (ps.t < 1) return fail(h, QAP_ESTATE, "the parent has run no iteration yet");
    return fold_core(h, l, s, ps.lb + px, child);
}

}  // extern "C"

namespace {

// The batched dual ascent shared by qap_batch_dual_ascent and
// qap_batch_dual_ascent_static.  With no_alloc the node table, prefix tables
// and stop counter go to the per-device static array (ws, ws_bytes), the
// iterations are launched directly (no captured graph: instantiating one
// allocates), the batched Z-LAP mapping is the tuned one if this process or
// the tune cache already holds it (else the rule-based one; every mapping
// gives the same results), and a handle whose trace has no room for the
// iterations is refused instead of grown.
// search_tune (the branch-and-bound's, one per search): Z-LAP mappings
// measured on this search's own tiles, by tile size.  The process-wide
// choice for a tile size is measured once, on the tiles of whatever batch
// first had that size, and suits other instances less well (a grid
// instance's tiles take the mappings' relative times elsewhere than a dense
// one's).  A batch whose Z-LAP work is at least kSearchTuneWork tile
// iterations (the measurement then costs about 2 % of it) is measured on
// its own tiles once per search and size; smaller batches, and later
// batches of a measured size, take the stored choice.  QAP_SEARCH_TUNE_WORK
// replaces the threshold (tests set it low so that small searches take
// this path).
constexpr double kSearchTuneWork = 1e8;

double search_tune_work()
{
    const char *e = std::getenv("QAP_SEARCH_TUNE_WORK");
    return (e && *e) ? std::atof(e) : kSearchTuneWork;
}

int batch_core(qap_handle *hs, int count, const qap_batch_params *bp, qap_batch_stats *st, bool no_alloc,
               char *ws, size_t ws_bytes, std::vector<DevScalars> *scal_out = nullptr,
               std::map<int, int> *search_tune = nullptr)
{
    if (count < 0 || (count > 0 && (!hs || !bp))) return fail(nullptr, QAP_EINVAL, "bad batch arguments");
    if (count == 0) return QAP_OK;
    if (bp->iters < 0 || bp->window < 0 || bp->window > 1000) return fail(hs[0], QAP_EINVAL, "bad batch params");
    {
        const int zl = bp->zlap_lanes;
        if (!(zl == 0 || zl == -1 || zl == -2 || zl == 8 || zl == 16 || zl == 32 || zl == 64))
            return fail(hs[0], QAP_EINVAL, "zlap_lanes must be 0, -1, -2, 8, 16, 32 or 64");
    }
    qap_ctx *h0 = hs[0];
    if (!h0) return QAP_EINVAL;
    hipStream_t stream = h0->stream;
    for (int b = 0; b < count; ++b) {
        if (!hs[b] || hs[b]->prm.device != h0->prm.device) return fail(h0, QAP_EINVAL, "handles on one device");
        if (hs[b]->n > 64) return fail(h0, QAP_EUNSUPPORTED, "n > 64 in a batch");
        if (hs[b]->prm.slow) return fail(h0, QAP_EUNSUPPORTED, "batched dual ascent is F1 only");
        if (hs[b]->Vt) return fail(h0, QAP_ESTATE, "a batched handle tracks multipliers");
        if (hs[b]->half) return fail(h0, QAP_EUNSUPPORTED, "batched dual ascent is FULL-scheme only");
        if (hs[b]->prm.two_phase) return fail(h0, QAP_EUNSUPPORTED, "batched dual ascent is F1 only");
        if (hs[b]->sa_on) return fail(h0, QAP_EUNSUPPORTED, "batched dual ascent runs without annealing");
    }
    auto t0 = std::chrono::steady_clock::now();
    HIPCHK(h0, hipSetDevice(h0->prm.device));
    {  // every handle's queued work first (each distinct stream once)
        std::vector<hipStream_t> streams;
        for (int b = 0; b < count; ++b)
            if (std::find(streams.begin(), streams.end(), hs[b]->stream) == streams.end())
                streams.push_back(hs[b]->stream);
        for (hipStream_t sm : streams) HIPCHK(h0, hipStreamSynchronize(sm));
    }
    // device copies (one allocation): node table, prefix tables, stop
    // counter, per-node stop flags, the handles' scalar-block addresses and
    // the gathered scalar blocks
    const size_t nb_bytes = round_up(sizeof(BNode) * count), pf_bytes = round_up(sizeof(long long) * (count + 1));
    const size_t fl_bytes = round_up(sizeof(int) * count), sp_bytes = round_up(sizeof(DevScalars *) * count);
    const size_t need = nb_bytes + 4 * pf_bytes + 256 + fl_bytes + sp_bytes + round_up(sizeof(DevScalars) * count);
    void *dmem = nullptr;
    if (no_alloc) {
        if (need > ws_bytes) return fail(h0, QAP_EINVAL, "batch tables exceed the static workspace");
        dmem = ws;
    } else {
        HIPCHK(h0, hipMalloc(&dmem, need));
    }
    std::unique_ptr<void, void (*)(void *)> guard(no_alloc ? nullptr : dmem, [](void *p) {
        if (p) (void)hipFree(p);
    });
    char *dp = (char *)dmem;
    DevScalars **dsptr = (DevScalars **)(dp + nb_bytes + 4 * pf_bytes + 256 + fl_bytes);
    DevScalars *dscal = (DevScalars *)(dp + nb_bytes + 4 * pf_bytes + 256 + fl_bytes + sp_bytes);
    // every handle's scalar block in one copy (gathered on the device)
    std::vector<DevScalars *> sptrs(count);
    for (int b = 0; b < count; ++b) sptrs[b] = hs[b]->S;
    std::vector<DevScalars> scal(count);
    auto gather_scalars = [&]() -> hipError_t {
        hipLaunchKernelGGL(k_bgather_scalars, dim3((count + 255) / 256), dim3(256), 0, stream, dsptr, count, dscal);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(scal.data(), dscal, sizeof(DevScalars) * count, hipMemcpyDeviceToHost, stream);
        return e == hipSuccess ? hipStreamSynchronize(stream) : e;
    };
    HIPCHK(h0, hipMemcpyAsync(dsptr, sptrs.data(), sizeof(DevScalars *) * count, hipMemcpyHostToDevice, stream));
    HIPCHK(h0, gather_scalars());
    // node descriptors of every handle; the tables hold the nodes still
    // running (a stopped node's jobs would only read its flag and leave)
    std::vector<BNode> all(count);
    std::vector<int> ids;
    std::vector<long long> work(count, 0);
    int mz = 1, my = 1, stopped0 = 0;
    for (int b = 0; b < count; ++b) {
        qap_ctx *h = hs[b];
        const DevScalars &s = scal[b];
        stopped0 += s.stopped ? 1 : 0;
        if (no_alloc) {
            if (s.t + bp->iters + 1 > h->trace_cap)
                return fail(h0, QAP_ESTATE, "a handle's bound trace has no room for the iterations (the "
                                            "allocating entry points grow it)");
        } else {
            int rc = ensure_trace(h, s.t + bp->iters + 1);
            if (rc != QAP_OK) return rc;
        }
        BNode &N = all[b];
        N.Z = h->Z;
        N.Yc = h->Yc;
        N.Py = h->Py;
        N.Xc = h->Xc;
        N.Px = h->Px;
        N.alpha = h->alpha;
        N.beta = h->beta;
        N.trace = h->trace;
        N.F = h->F;
        N.D = h->D;
        N.B = h->B;
        N.xperm = h->xperm;
        N.bestperm = h->bestperm;
        N.S = h->S;
        N.bins = h->bins;
        N.triples = h->triples;
        N.T = h->T;
        N.n = h->n;
        N.m = h->m;
        N.ntri = h->ntriples;
        N.nb = (h->n + SB - 1) / SB;
        N.integer_data = h->integer_data ? 1 : 0;
        N.trace_cap = h->trace_cap;
        N.offset = h->offset;
        N.min_gap = h->prm.min_gap;
        N.kz = h->kz;
        N.okz = h->okz;
        N.ky2 = h->ky2;
        N.kx3 = h->kx3;
        N.phi = h->phi;
        N.oky = h->oky;
        N.okx = h->okx;
        N.phy = h->phy;
        N.ophy = h->ophy;
        work[b] = h->T * (long long)h->m * h->m + h->T + (long long)h->n * h->n;
        if (!s.stopped) {
            ids.push_back(b);
            mz = std::max(mz, h->m);
            my = std::max(my, h->n - 1);
        }
    }
    BNode *dnodes = (BNode *)dp;
    long long *dzl = (long long *)(dp + nb_bytes), *dyl = (long long *)(dp + nb_bytes + pf_bytes);
    long long *dsw = (long long *)(dp + nb_bytes + 2 * pf_bytes), *dsc = (long long *)(dp + nb_bytes + 3 * pf_bytes);
    int *dnstop = (int *)(dp + nb_bytes + 4 * pf_bytes);
    int *dflags = (int *)(dp + nb_bytes + 4 * pf_bytes + 256);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, stream, (double *)dnstop, (size_t)1, 0.0);  // zeroes the counter
    HIPCHK(h0, hipGetLastError());
    // the tables of the nodes in ids; their host copies stay unchanged until
    // the stream has drained (the next poll)
    std::vector<BNode> nodes;
    std::vector<long long> zl, yl, sw, sc;
    int cur = 0;
    auto upload = [&]() -> hipError_t {
        cur = (int)ids.size();
        nodes.resize(cur);
        zl.assign(cur + 1, 0);
        yl.assign(cur + 1, 0);
        sw.assign(cur + 1, 0);
        sc.assign(cur + 1, 0);
        for (int i = 0; i < cur; ++i) {
            const BNode &N = all[ids[i]];
            nodes[i] = N;
            zl[i + 1] = zl[i] + N.T;
            yl[i + 1] = yl[i] + (long long)N.n * N.n;
            sw[i + 1] = sw[i] + (long long)N.ntri * N.nb * N.nb * N.nb;
            sc[i + 1] = sc[i] + N.T + (long long)N.n * N.n;
        }
        if (cur == 0) return hipSuccess;
        hipError_t e;
        if ((e = hipMemcpyAsync(dnodes, nodes.data(), sizeof(BNode) * cur, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return e;
        const size_t pb = sizeof(long long) * (cur + 1);
        if ((e = hipMemcpyAsync(dzl, zl.data(), pb, hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(dyl, yl.data(), pb, hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(dsw, sw.data(), pb, hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
        return hipMemcpyAsync(dsc, sc.data(), pb, hipMemcpyHostToDevice, stream);
    };
    HIPCHK(h0, upload());
    BatchPrefix pf{dzl, dyl, dsw, dsc};
    BatchCtl ctl{bp->ub_cut, bp->min_improve, bp->window, count, dnstop};
    // measured once per tile size (looked up only, without allocating)
    if ((bp->zlap_lanes > 0 && bp->zlap_lanes < mz) || (bp->zlap_lanes < 0 && mz > 32))
        return fail(h0, QAP_EINVAL, "zlap_lanes does not hold the batch's largest tile");
    // real tiles for a first timing of the mappings at this tile size: a
    // node of the largest m whose z holds reduced costs (it has iterated, or
    // it was folded from its parent), else none (synthetic tiles)
    const double *tune_src = nullptr;
    long long tune_tiles_n = 0;
    for (int b : ids)
        if (hs[b]->m == mz && (scal[b].t >= 1 || hs[b]->folded)) {
            tune_src = hs[b]->Z;
            tune_tiles_n = hs[b]->T;
            break;
        }
    int Lz;
    if (cur == 0)
        Lz = -1;
    else if (bp->zlap_lanes != 0)
        Lz = bp->zlap_lanes;
    else if (no_alloc)
        Lz = known_batch_lanes(h0->prm.device, mz);
    else if (search_tune && search_tune->count(mz))
        Lz = (*search_tune)[mz];
    else if (search_tune && tune_src && (double)zl[cur] * bp->iters >= search_tune_work())
        Lz = (*search_tune)[mz] = measure_bzlap(stream, mz, tune_src, tune_tiles_n).lanes;
    else
        Lz = tuned_batch_lanes(h0->prm.device, stream, mz, tune_src, tune_tiles_n);
    const int Ly = my <= 8 ? 8 : my <= 16 ? 16 : my <= 32 ? 32 : 64;
    auto launch_all = [&]() -> hipError_t {
        hipError_t e;
        const int count = cur;  // the nodes in the tables
        if (sw[count] > 0) {
            const unsigned grid = (unsigned)((sw[count] + 7) / 8 * 8);  // k_bsweep deals eighths to the XCDs
            hipLaunchKernelGGL(k_bsweep, dim3(grid), dim3(256), 0, stream, dnodes, pf, count);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        const unsigned sb = (unsigned)std::min<long long>((sc[count] + 255) / 256, 65535);
        hipLaunchKernelGGL(k_bscale, dim3(sb), dim3(256), 0, stream, dnodes, pf, count);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        {
            const size_t per = ((size_t)mz * mz + 2 * mz) * sizeof(double);
            int G = 256 / Lz;
            while (G > 1 && (size_t)G * per > 65536) --G;
            const unsigned blocks = (unsigned)((zl[count] + G - 1) / G);
#define QAP_BZ(LL)                                                                                              \
    if (Lz == LL) hipLaunchKernelGGL((k_bzlap<LL>), dim3(blocks), dim3(G * LL), G * per, stream, dnodes, pf, count, mz);
            QAP_BZ(8) QAP_BZ(16) QAP_BZ(32) QAP_BZ(64)
#undef QAP_BZ
            if (Lz == -1)  // one tile per wavefront
                hipLaunchKernelGGL(k_bzlap_s, dim3((unsigned)zl[count]), dim3(64), per, stream, dnodes, pf, count);
            if (Lz == -2)  // two tiles per wavefront (every node's tile count is even)
                hipLaunchKernelGGL(k_bzlap_s2, dim3((unsigned)(zl[count] / 2)), dim3(64), 2 * per, stream, dnodes, pf,
                                   count);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            const size_t per = ((size_t)my * my + 2 * my) * sizeof(double);
            int G = 256 / Ly;
            while (G > 1 && (size_t)G * per > 65536) --G;
            const unsigned blocks = (unsigned)((yl[count] + G - 1) / G);
#define QAP_BY(LL)                                                                                              \
    if (Ly == LL) hipLaunchKernelGGL((k_bylap<LL>), dim3(blocks), dim3(G * LL), G * per, stream, dnodes, pf, count, my);
            QAP_BY(8) QAP_BY(16) QAP_BY(32) QAP_BY(64)
#undef QAP_BY
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_bxlap, dim3(count), dim3(64), 0, stream, dnodes, ctl);
        return hipGetLastError();
    };
    int compactions = 0;
    if (bp->iters > 0 && cur > 0) {
        // one captured graph of the tables' kernels, replayed; the legacy
        // null stream cannot be captured, there every replay launches the
        // kernels
        hipGraphExec_t ge = nullptr;
        const bool use_graph = stream != nullptr && !no_alloc;
        auto capture = [&]() -> std::string {
            hipGraph_t g = nullptr;
            hipError_t be = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (be != hipSuccess) return std::string("batch capture: ") + hipGetErrorString(be);
            hipError_t le = launch_all();
            hipError_t ce = hipStreamEndCapture(stream, &g);
            if (le != hipSuccess) return std::string("batch launch: ") + hipGetErrorString(le);
            if (ce != hipSuccess) return std::string("batch capture: ") + hipGetErrorString(ce);
            hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                ge = nullptr;
                return std::string("batch graph: ") + hipGetErrorString(ie);
            }
            return std::string();
        };
        if (use_graph) {
            const std::string err = capture();
            if (!err.empty()) return fail(h0, QAP_EDEVICE, err);
        }
        // replays; every kPoll of them the host reads how many nodes have
        // stopped and ends the batch once all have.  When nodes stopped since
        // the last look, it reads which, and once they hold at least an
        // eighth of the tables' work it drops them from the tables (and
        // captures the smaller graph): a node's arithmetic does not depend
        // on which other nodes share its launches.
        constexpr int kPoll = 4;
        int seen = 0;
        std::vector<int> flags;
        std::string err;
        for (int it = 0; it < bp->iters && err.empty(); ++it) {
            hipError_t e2 = ge ? hipGraphLaunch(ge, stream) : launch_all();
            if (e2 == hipSuccess && (it + 1) % kPoll == 0 && it + 1 < bp->iters) {
                int ns = 0;
                e2 = hipMemcpyAsync(&ns, dnstop, sizeof(int), hipMemcpyDeviceToHost, stream);
                if (e2 == hipSuccess) e2 = hipStreamSynchronize(stream);
                if (e2 == hipSuccess && stopped0 + ns >= count) break;
                if (e2 == hipSuccess && ns > seen) {
                    seen = ns;
                    flags.assign(cur, 0);
                    hipLaunchKernelGGL(k_bstopped, dim3((cur + 255) / 256), dim3(256), 0, stream, dnodes, cur, dflags);
                    e2 = hipGetLastError();
                    if (e2 == hipSuccess)
                        e2 = hipMemcpyAsync(flags.data(), dflags, sizeof(int) * cur, hipMemcpyDeviceToHost, stream);
                    if (e2 == hipSuccess) e2 = hipStreamSynchronize(stream);
                    long long w_all = 0, w_live = 0;
                    std::vector<int> keep;
                    for (int i = 0; e2 == hipSuccess && i < cur; ++i) {
                        w_all += work[ids[i]];
                        if (!flags[i]) {
                            keep.push_back(ids[i]);
                            w_live += work[ids[i]];
                        }
                    }
                    if (e2 == hipSuccess && 8 * (w_all - w_live) >= w_all) {
                        // the stream has drained: no replay reads the old
                        // tables or the old exec's arguments any more
                        if (ge) (void)hipGraphExecDestroy(ge);
                        ge = nullptr;
                        ids.swap(keep);
                        ++compactions;
                        e2 = upload();
                        if (e2 == hipSuccess && cur == 0) break;
                        if (e2 == hipSuccess && use_graph) err = capture();
                    }
                }
            }
            if (e2 != hipSuccess) err = std::string("batch replay: ") + hipGetErrorString(e2);
        }
        // the graph exec owns the kernel arguments of its nodes; replays
        // still in the stream's queue read them when they are dispatched,
        // so the exec is destroyed only after the stream has drained
        const hipError_t se = hipStreamSynchronize(stream);
        if (ge) (void)hipGraphExecDestroy(ge);
        if (!err.empty()) return fail(h0, QAP_EDEVICE, err);
        if (se != hipSuccess) return fail(h0, QAP_EDEVICE, std::string("batch sync: ") + hipGetErrorString(se));
    }
    HIPCHK(h0, gather_scalars());
    if (st) {
        std::memset(st, 0, sizeof(*st));
        for (int b = 0; b < count; ++b) {
            const DevScalars &s = scal[b];
            st->iterations += s.t;
            st->stopped += s.stopped ? 1 : 0;
            st->fathomed += s.reason == 1 ? 1 : 0;
            st->window_stops += s.reason == 2 ? 1 : 0;
        }
        st->compactions = compactions;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    for (int b = 0; b < count; ++b) hs[b]->t_host = scal[b].t;
    if (scal_out) scal_out->swap(scal);
    return QAP_OK;
}

}  // namespace

extern "C" {

int qap_batch_dual_ascent(qap_handle *hs, int count, const qap_batch_params *bp, qap_batch_stats *st)
{
    return batch_core(hs, count, bp, st, false, nullptr, 0);
}

int qap_batch_dual_ascent_static(qap_handle *hs, int count, const qap_batch_params *bp, qap_batch_stats *st)
{
    if (count < 0 || count > QAP_BATCH_STATIC_MAX_NODES || (count > 0 && (!hs || !bp)))
        return fail(nullptr, QAP_EINVAL, "bad batch arguments (count must be 0..QAP_BATCH_STATIC_MAX_NODES)");
    if (count == 0) return QAP_OK;
    if (!hs[0]) return QAP_EINVAL;
    char *ws = nullptr;
    const int rc = static_workspace(hs[0], &ws);
    if (rc != QAP_OK) return rc;
    return batch_core(hs, count, bp, st, true, ws, QAP_BATCH_STATIC_BYTES);
}

int qap_node_status(qap_handle h, int *t, double *lb, double *ub, int *stopped, int *reason)
{
    if (!h) return QAP_EINVAL;
    DevScalars s{};
    HIPCHK(h, hipMemcpyAsync(&s, h->S, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (t) *t = s.t;
    if (lb) *lb = s.lb;
    if (ub) *ub = s.ub;
    if (stopped) *stopped = s.stopped;
    if (reason) *reason = s.reason;
    return QAP_OK;
}

// The QAP left when the facilities with fixed[i] >= 0 sit at those
// locations: F and D restricted to the free facilities `fac` and free
// locations `loc`, b'_ac = b_{fac[a],loc[c]} + sum over fixed i of
// (f_{fac[a],i} d_{loc[c],fixed[i]} + f_{i,fac[a]} d_{fixed[i],loc[c]}), and the
// constant offset = sum over fixed i of b_{i,fixed[i]} + sum over fixed i, j of
// f_ij d_{fixed[i],fixed[j]}.  Its cost plus the offset is the full cost of
// every completion.
void restricted_qap(const qap_ctx *h, const std::vector<int> &fac, const std::vector<int> &loc,
                    const std::vector<int> &fixed, std::vector<double> &Fc, std::vector<double> &Dc,
                    std::vector<double> &Bc, double &offset)
{
    const int n = h->n, k = (int)fac.size();
    const double *F = h->hF.data(), *D = h->hD.data(), *B = h->hB.data();
    Fc.assign((size_t)k * k, 0.0);
    Dc.assign((size_t)k * k, 0.0);
    Bc.assign((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            Fc[a * k + c] = F[fac[a] * n + fac[c]];
            Dc[a * k + c] = D[loc[a] * n + loc[c]];
            double b = B[fac[a] * n + loc[c]];
            for (int i = 0; i < n; ++i)
                if (fixed[i] >= 0)
                    b = (b + F[fac[a] * n + i] * D[loc[c] * n + fixed[i]]) + F[i * n + fac[a]] * D[fixed[i] * n + loc[c]];
            Bc[a * k + c] = b;
        }
    double off = 0.0;
    for (int i = 0; i < n; ++i) {
        if (fixed[i] < 0) continue;
        off += B[i * n + fixed[i]];
        for (int j = 0; j < n; ++j)
            if (fixed[j] >= 0) off += F[i * n + j] * D[fixed[i] * n + fixed[j]];
    }
    offset = off;
}

int qap_bnb_solve(qap_handle h, const qap_bnb_params *p, int32_t *perm_out, double *obj_out, qap_bnb_stats *st)
{
    if (!h || !perm_out || !obj_out) return QAP_EINVAL;
    if (h->half) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound is FULL-scheme only");
    if (h->prm.two_phase) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound is F1 only");
    if (h->sa_on) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound runs without annealing");
    if (h->prm.slow) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound is F1 only");
    qap_bnb_params P{};
    if (p) {
        P = *p;
    } else {
        P.batch = 256;
        P.node_iters = 100;
        P.window = 25;
        P.root_iters = 0;
        P.min_improve = 2e-4;
        P.ub0 = HUGE_VAL;
        P.enum_below = 3;
        P.rule = 3;
        P.depth_cap = 0;
        P.symmetry = 0;
    }
    if (P.batch < 1 || P.node_iters < 1 || P.window < 0 || P.window > 1000 || P.enum_below < 3 ||
        !(P.min_improve >= 0.0) || P.rule != 3 || P.depth_cap < 0 || P.symmetry < 0 || P.symmetry > 1)
        return fail(h, QAP_EINVAL, "bad branch-and-bound parameters");
    if (P.root_iters <= 0) P.root_iters = P.node_iters;
    const int n = h->n;
    if (n > 24) return fail(h, QAP_EUNSUPPORTED, "branch-and-bound supports n <= 24");
    auto t0 = std::chrono::steady_clock::now();
    const std::vector<int> order = rule3_order(n, h->hF.data());
    // symmetry elimination: the non-identity location automorphisms
    std::vector<std::vector<int>> autos;
    if (P.symmetry) {
        autos = location_automorphisms(n, h->hD.data(), h->hB.data(), 4096);
        if (!autos.empty()) autos.erase(autos.begin());  // the identity
    }
    long long sym_skipped = 0;
    const bool integer_data = h->integer_data;
    double UB = P.ub0;
    std::vector<int> best(n, -1);
    long long nodes_done = 0, da_iters = 0, batches = 0, enumerated = 0;
    std::map<int, int> search_tune;  // Z-LAP mappings measured on this search's tiles
    double node_bytes = 0.0;
    // node handles take their arenas from the pool unless h has an allocator
    // of its own (children inherit the parameters of their parent); declared
    // before every handle of the search, so it outlives them
    NodeArenaPool pool;
    qap_params cprm = h->prm;
    if (!cprm.alloc) {
        cprm.alloc = NodeArenaPool::alloc;
        cprm.free_fn = NodeArenaPool::release;
        cprm.alloc_ctx = &pool;
    }

    struct Node {
        std::shared_ptr<qap_ctx> parent;  // materialised parent state (shared by siblings)
        int l = -1, s = -1;               // fold of the parent, or -1 for the root
        int depth = 0;
        double lb_hint = -HUGE_VAL;       // parent bound + pi_x[l,s]
        std::vector<int> fac, loc, fixed;
    };
    auto destroy = [](qap_ctx *c) { qap_destroy(c); };
    auto update_ub = [&](double cost, const std::vector<int> &perm) {
        if (cost < UB) {
            UB = cost;
            best = perm;
        }
    };
    // exact completion of a node with at most enum_below free facilities
    auto enumerate = [&](const Node &nd) {
        const int k = (int)nd.fac.size();
        std::vector<int> a(k);
        for (int t = 0; t < k; ++t) a[t] = t;
        std::vector<int> perm = nd.fixed;
        do {
            for (int t = 0; t < k; ++t) perm[nd.fac[t]] = nd.loc[a[t]];
            update_ub(full_cost(h, perm), perm);
            ++enumerated;
        } while (std::next_permutation(a.begin(), a.end()));
    };

    std::vector<Node> stack;
    {
        Node root;
        root.depth = 0;
        for (int i = 0; i < n; ++i) {
            root.fac.push_back(i);
            root.loc.push_back(i);
        }
        root.fixed.assign(n, -1);
        if (n <= P.enum_below) {
            enumerate(root);
            ++nodes_done;
        } else {
            stack.push_back(root);
        }
    }
    int rc = QAP_OK;
    while (!stack.empty() && rc == QAP_OK) {
        // next batch: the top of the stack (deepest, lowest location first)
        std::vector<Node> batch;
        while (!stack.empty() && (int)batch.size() < P.batch) {
            Node nd = std::move(stack.back());
            stack.pop_back();
            if (fathomed_host(nd.lb_hint, UB, integer_data)) {
                ++nodes_done;
                continue;
            }
            batch.push_back(std::move(nd));
        }
        if (batch.empty()) continue;
        std::vector<std::shared_ptr<qap_ctx>> ctxs;
        std::vector<qap_handle> hs;
        for (auto &nd : batch) {
            qap_ctx *c = nullptr;
            if (nd.l < 0) {
                rc = create_ctx(n, h->hF.data(), h->hD.data(), h->hB.data(), cprm, 0.0, h->stream, true, &c);
                if (rc != QAP_OK) h->err = g_init_error;
            } else if (!nd.parent) {
                // past the depth cap: the restricted QAP of the node, from scratch
                std::vector<double> Fc, Dc, Bc;
                double off = 0.0;
                restricted_qap(h, nd.fac, nd.loc, nd.fixed, Fc, Dc, Bc, off);
                rc = create_ctx((int)nd.fac.size(), Fc.data(), Dc.data(), Bc.data(), cprm, off, h->stream, true,
                                &c);
                if (rc != QAP_OK)
                    h->err = g_init_error;
                else if ((rc = upload_scalars(c, off)) != QAP_OK)  // the bound counts the fixed part too
                    h->err = c->err;
            } else {
                // the child's starting bound is the parent's bound plus
                // pi_x[l][s], read after the parent's batch (lb_hint)
                rc = fold_core(nd.parent.get(), nd.l, nd.s, nd.lb_hint, &c);
                if (rc != QAP_OK) h->err = nd.parent->err;
            }
            if (rc != QAP_OK) break;
            nd.parent.reset();  // release the parent once its last child is built
            ctxs.emplace_back(c, destroy);
            hs.push_back(c);
        }
        if (rc != QAP_OK) break;
        const int iters = (batch.size() == 1 && batch[0].depth == 0) ? P.root_iters : P.node_iters;
        qap_batch_params bp{iters, P.window, P.min_improve, UB};
        // (the nodes' scalar blocks come back with the batch, in one copy)
        std::vector<DevScalars> sv;
        rc = batch_core(hs.data(), (int)hs.size(), &bp, nullptr, false, nullptr, 0, &sv, &search_tune);
        if (rc != QAP_OK) {
            h->err = hs[0]->err;
            break;
        }
        ++batches;
        // incumbents first, then branching with the improved UB
        for (size_t b = 0; b < hs.size(); ++b) {
            qap_ctx *c = hs[b];
            da_iters += sv[b].t;
            {
                const double nn = c->n, T1 = nn * nn * (nn - 1) * (nn - 1), V1 = T1 * (nn - 2) * (nn - 2);
                node_bytes += sv[b].t * 8.0 * (4.0 * V1 + 8.0 * T1 + 10.0 * nn * nn);
            }
            std::vector<int> lp(c->n);
            if (hipMemcpy(lp.data(), c->bestperm, sizeof(int) * c->n, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(h, QAP_EDEVICE, "reading node assignment failed");
                break;
            }
            if (sv[b].ub < HUGE_VAL) {
                std::vector<int> perm = batch[b].fixed;
                for (int a = 0; a < c->n; ++a) perm[batch[b].fac[a]] = batch[b].loc[lp[a]];
                update_ub(full_cost(h, perm), perm);
            }
        }
        if (rc != QAP_OK) break;
        std::vector<Node> pushes;
        for (size_t b = 0; b < hs.size(); ++b) {
            ++nodes_done;
            Node &nd = batch[b];
            if (fathomed_host(sv[b].lb, UB, integer_data)) continue;
            if (sv[b].t < 1) {  // (every batch runs at least one iteration of a fresh node)
                rc = fail(h, QAP_ESTATE, "a node to branch on has run no iteration");
                break;
            }
            const int nl = (int)nd.fac.size();
            const int f = order[nd.depth];
            int l = -1;
            for (int t = 0; t < nl; ++t)
                if (nd.fac[t] == f) l = t;
            std::vector<double> pxr(nl);
            if (hipMemcpy(pxr.data(), hs[b]->Px + (size_t)l * nl, sizeof(double) * nl, hipMemcpyDeviceToHost) !=
                hipSuccess) {
                rc = fail(h, QAP_EDEVICE, "reading pi_x failed");
                break;
            }
            // automorphisms that keep every placed facility where it is: a
            // child whose location one of them maps lower is equivalent to
            // that lower child (same costs below it) and is not built
            std::vector<const std::vector<int> *> stab;
            for (const auto &a : autos) {
                bool fixes = true;
                for (int i = 0; fixes && i < n; ++i)
                    if (nd.fixed[i] >= 0 && a[nd.fixed[i]] != nd.fixed[i]) fixes = false;
                if (fixes) stab.push_back(&a);
            }
            std::vector<Node> kids;
            for (int s = 0; s < nl; ++s) {
                bool dominated = false;
                for (const auto *a : stab)
                    if ((*a)[nd.loc[s]] < nd.loc[s]) dominated = true;
                if (dominated) {
                    ++sym_skipped;
                    continue;
                }
                const double lbc = sv[b].lb + pxr[s];
                if (fathomed_host(lbc, UB, integer_data)) continue;
                Node k;
                k.depth = nd.depth + 1;
                k.l = l;
                k.s = s;
                k.lb_hint = lbc;
                for (int t = 0; t < nl; ++t)
                    if (t != l) k.fac.push_back(nd.fac[t]);
                for (int t = 0; t < nl; ++t)
                    if (t != s) k.loc.push_back(nd.loc[t]);
                k.fixed = nd.fixed;
                k.fixed[f] = nd.loc[s];
                if (nl - 1 <= P.enum_below) {
                    enumerate(k);
                    ++nodes_done;
                    continue;
                }
                if (P.depth_cap == 0 || k.depth <= P.depth_cap) k.parent = ctxs[b];
                kids.push_back(std::move(k));
            }
            for (auto &k : kids) pushes.push_back(std::move(k));
        }
        // pushes is in priority order (batch order, then ascending location):
        // push it reversed so that its first entry ends on top
        for (auto it = pushes.rbegin(); it != pushes.rend(); ++it) stack.push_back(std::move(*it));
    }
    if (rc != QAP_OK) return rc;
    if (!(UB < HUGE_VAL)) return fail(h, QAP_ESTATE, "no incumbent below ub0");
    for (int i = 0; i < n; ++i) perm_out[i] = best[i];
    *obj_out = UB;
    if (st) {
        st->nodes = nodes_done;
        st->da_iters = da_iters;
        st->batches = batches;
        st->enumerated = enumerated;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        st->symmetric_skipped = sym_skipped;
        st->automorphisms = (long long)autos.size() + 1;
        st->node_bytes = node_bytes;
    }
    return QAP_OK;
}

}  // extern "C"
