// tune_host.hpp -- the LAP-mapping autotuner.
//
// Every Z-LAP mapping (one LAP per wavefront; two per wavefront when
// m <= 32; L-lane groups with C columns per lane, L*C >= m) computes bitwise
// the same LAP results, so the mapping decides only the speed.  For a LAP
// size m the tuner times each mapping that can hold m with the Z-LAP kernels
// themselves on a fixed synthetic batch of tiles and keeps the fastest.  The
// batched branch-and-bound Z-LAP kernel (lane groups, or one tile per
// wavefront) is chosen the same way on a one-node batch.  Choices are kept
// per process and, when the environment variable QAP_TUNE_CACHE names a
// file, in that JSON file, keyed by the GPU architecture, the kernel, m and
// a revision number of the kernels and candidates (bumped when they change).
//
// The synthetic tiles hold integers 0..99 from a hash of the entry index:
// fresh LAPs of the instances' cost scale.  Later Z-LAPs see reduced costs
// with fewer Dijkstra steps; the ranking of mappings is taken to carry over.
#pragma once
#include <cstdlib>
#include <map>
#include <mutex>

#include "batch.hpp"

namespace qap {

__global__ void k_tune_fill(double *__restrict__ a, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long x = (i + 1) * 0x9E3779B97F4A7C15ull;  // splitmix64 finalizer of the index
        x ^= x >> 30;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 27;
        x *= 0x94D049BB133111EBull;
        x ^= x >> 31;
        a[i] = (double)(x % 100ull);
    }
}

}  // namespace qap

namespace {

constexpr int kTuneRev = 3;                          // revision of the tuned kernels and candidates
constexpr long long kTuneTiles = 32768;              // synthetic tiles per timing (fewer for large m)
constexpr size_t kTuneBytes = (size_t)256 << 20;     // cap on the synthetic tile bytes
constexpr int kTuneReps = 3;                         // timed launches per mapping, after one warm-up

struct TuneChoice {
    int lanes, cols;
    double us;  // best launch time over the synthetic batch; < 0: not measured (rule-based fallback)
};

std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;  // this process's choices

std::string tune_key(int device, const char *kernel, int m)
{
    hipDeviceProp_t prop{};
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%s/m%d/r%d", arch.c_str(), kernel, m, kTuneRev);
    return buf;
}

// The cache file holds one JSON object: {"<key>": [lanes, cols, microseconds], ...}.
std::map<std::string, TuneChoice> read_tune_file(const char *path)
{
    std::map<std::string, TuneChoice> out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        TuneChoice c{0, 0, 0.0};
        if (std::sscanf(text.c_str() + end + 1, " : [ %d , %d , %lf ]", &c.lanes, &c.cols, &c.us) == 3)
            out[text.substr(pos + 1, end - pos - 1)] = c;
        pos = end + 1;
    }
    return out;
}

void write_tune_file(const char *path, const std::map<std::string, TuneChoice> &entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : entries) {
        ++i;
        std::fprintf(f, "  \"%s\": [%d, %d, %.3f]%s\n", kv.first.c_str(), kv.second.lanes, kv.second.cols,
                     kv.second.us, i < entries.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path);
}

// The choice for key: this process's, else the cache file's, else measure()'s
// (recorded in both when it measured something).
template <class Measure>
TuneChoice tuned_choice(const std::string &key, Measure measure)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const char *path = std::getenv("QAP_TUNE_CACHE");
    const bool use_file = path && *path;
    std::map<std::string, TuneChoice> file;
    if (use_file) file = read_tune_file(path);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) {
        const auto fit = file.find(key);
        it = g_tune.emplace(key, fit != file.end() ? fit->second : measure()).first;
    }
    if (use_file && it->second.us >= 0.0 && file.find(key) == file.end()) {
        file[key] = it->second;
        write_tune_file(path, file);
    }
    return it->second;
}

// Device scratch for one tuning run, released on every path.
struct TuneScratch {
    std::vector<void *> ptrs;
    void *get(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
    ~TuneScratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

// Best (minimum) time in microseconds of launch() over the synthetic tiles,
// each launch on a fresh copy of them; < 0 on any HIP error.
template <class Launch>
double time_launches(hipStream_t stream, double *work, const double *src, size_t count, Launch launch)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double best = -1.0;
    for (int rep = 0; rep <= kTuneReps; ++rep) {
        if (hipMemcpyAsync(work, src, sizeof(double) * count, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            hipEventRecord(e0, stream) != hipSuccess || launch() != hipSuccess ||
            hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            best = -1.0;
            break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = -1.0;
            break;
        }
        if (rep > 0 && (best < 0.0 || 1e3 * ms < best)) best = 1e3 * ms;  // rep 0 warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

long long tune_tiles(int m) { return std::max(1024ll, std::min(kTuneTiles, (long long)(kTuneBytes / (sizeof(double) * m * m)))); }

// Fills src with the synthetic tiles and zeroes the step counters and
// scalars (stopped = 0); false on a HIP error.
bool tune_inputs(hipStream_t stream, double *src, size_t count, DevScalars *S, unsigned long long *bins)
{
    hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, stream, src, count);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, stream, (double *)S, sizeof(DevScalars) / sizeof(double), 0.0);
    hipLaunchKernelGGL(k_fill, dim3(16), dim3(256), 0, stream, (double *)bins, (size_t)kStepBins, 0.0);
    return hipGetLastError() == hipSuccess;
}

// Fastest Z-LAP mapping for tiles of size m (the mappings of pick_zlap's
// explicit requests); falls back to the rule-based choice without timing.
TuneChoice measure_zlap(hipStream_t stream, int m, int zlap_waves)
{
    TuneChoice best{0, 0, -1.0};
    pick_zlap(m, 0, 0, best.lanes, best.cols);
    std::vector<std::pair<int, int>> cands{{-1, 1}};
    if (m <= 32) cands.push_back({-2, 1});
    const int groups[][2] = {{8, 1}, {16, 1}, {32, 1}, {64, 1}, {8, 2}, {16, 2}, {32, 2}, {8, 4}, {16, 4}};
    for (const auto &g : groups)
        if (g[0] * g[1] >= m) cands.push_back({g[0], g[1]});
    const long long N = tune_tiles(m);
    const size_t count = (size_t)N * m * m;
    TuneScratch mem;
    double *src = (double *)mem.get(sizeof(double) * count), *work = (double *)mem.get(sizeof(double) * count);
    double *Yc = (double *)mem.get(sizeof(double) * N);
    DevScalars *S = (DevScalars *)mem.get(256);
    unsigned long long *bins = (unsigned long long *)mem.get(sizeof(unsigned long long) * kStepBins);
    if (!src || !work || !Yc || !S || !bins || !tune_inputs(stream, src, count, S, bins)) return best;
    qap_ctx t;  // a view of the scratch as a context: only the Z-LAP launch fields are used
    t.m = m;
    t.T = N;
    t.Z = work;
    t.Yc = Yc;
    t.S = S;
    t.bins = bins;
    t.stream = stream;
    t.zlap_waves = zlap_waves;
    for (const auto &c : cands) {
        t.zl = c.first;
        t.zc = c.second;
        const double us = time_launches(stream, work, src, count, [&] { return launch_zlap(&t); });
        if (us >= 0.0 && (best.us < 0.0 || us < best.us)) best = TuneChoice{c.first, c.second, us};
    }
    (void)hipStreamSynchronize(stream);
    return best;
}

// Fastest batched Z-LAP kernel for tiles of size m (one node): lane groups
// of 8..64 (k_bzlap<L>, L >= m), or one or two tiles per wavefront
// (k_bzlap_s, lanes -1, and k_bzlap_s2, lanes -2; m <= 32); falls back to
// the smallest group that holds m.  real (nullable): real_tiles tiles of
// size m of a node about to be solved, timed instead of the synthetic ones
// when there are enough of them (a node's tiles after a few iterations
// solve in far fewer Dijkstra steps than random ones, and the mappings'
// order can differ between the two).
TuneChoice measure_bzlap(hipStream_t stream, int m, const double *real = nullptr, long long real_tiles = 0)
{
    TuneChoice best{m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64, 1, -1.0};
    const bool use_real = real && real_tiles >= 1024;
    const long long N = use_real ? std::min(tune_tiles(m), real_tiles) / 2 * 2 : tune_tiles(m);
    const size_t count = (size_t)N * m * m;
    TuneScratch mem;
    double *src = (double *)mem.get(sizeof(double) * count), *work = (double *)mem.get(sizeof(double) * count);
    double *Yc = (double *)mem.get(sizeof(double) * N);
    DevScalars *S = (DevScalars *)mem.get(256);
    unsigned long long *bins = (unsigned long long *)mem.get(sizeof(unsigned long long) * kStepBins);
    BNode *dnode = (BNode *)mem.get(sizeof(BNode));
    long long *dzl = (long long *)mem.get(2 * sizeof(long long));
    if (!src || !work || !Yc || !S || !bins || !dnode || !dzl || !tune_inputs(stream, src, count, S, bins))
        return best;
    if (use_real && hipMemcpyAsync(src, real, sizeof(double) * count, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return best;
    BNode node{};
    node.Z = work;
    node.Yc = Yc;
    node.S = S;
    node.bins = bins;
    node.T = N;
    node.m = m;
    const long long zl[2] = {0, N};
    if (hipMemcpyAsync(dnode, &node, sizeof(node), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(dzl, zl, sizeof(zl), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return best;
    BatchPrefix pf{dzl, dzl, dzl, dzl};  // only the tile prefix is read by k_bzlap
    const size_t per = ((size_t)m * m + 2 * m) * sizeof(double);
    for (int L : {8, 16, 32, 64}) {
        if (L < m) continue;
        int G = 256 / L;
        while (G > 1 && (size_t)G * per > 65536) --G;
        const unsigned blocks = (unsigned)((N + G - 1) / G);
        auto launch = [&]() -> hipError_t {
            if (L == 8) hipLaunchKernelGGL((k_bzlap<8>), dim3(blocks), dim3(G * 8), G * per, stream, dnode, pf, 1, m);
            if (L == 16) hipLaunchKernelGGL((k_bzlap<16>), dim3(blocks), dim3(G * 16), G * per, stream, dnode, pf, 1, m);
            if (L == 32) hipLaunchKernelGGL((k_bzlap<32>), dim3(blocks), dim3(G * 32), G * per, stream, dnode, pf, 1, m);
            if (L == 64) hipLaunchKernelGGL((k_bzlap<64>), dim3(blocks), dim3(G * 64), G * per, stream, dnode, pf, 1, m);
            return hipGetLastError();
        };
        const double us = time_launches(stream, work, src, count, launch);
        if (us >= 0.0 && (best.us < 0.0 || us < best.us)) best = TuneChoice{L, 1, us};
    }
    if (m <= 32) {
        auto launch = [&]() -> hipError_t {
            hipLaunchKernelGGL(k_bzlap_s, dim3((unsigned)N), dim3(64), per, stream, dnode, pf, 1);
            return hipGetLastError();
        };
        const double us = time_launches(stream, work, src, count, launch);
        if (us >= 0.0 && (best.us < 0.0 || us < best.us)) best = TuneChoice{-1, 1, us};
        auto launch2 = [&]() -> hipError_t {
            hipLaunchKernelGGL(k_bzlap_s2, dim3((unsigned)(N / 2)), dim3(64), 2 * per, stream, dnode, pf, 1);
            return hipGetLastError();
        };
        const double us2 = time_launches(stream, work, src, count, launch2);
        if (us2 >= 0.0 && (best.us < 0.0 || us2 < best.us)) best = TuneChoice{-2, 1, us2};
    }
    (void)hipStreamSynchronize(stream);
    return best;
}

// The handle's Z-LAP mapping when it was created with automatic mapping.
void tune_handle_zlap(qap_ctx *h)
{
    const TuneChoice c = tuned_choice(tune_key(h->prm.device, "zlap", h->m),
                                      [&] { return measure_zlap(h->stream, h->m, h->zlap_waves); });
    h->zl = c.lanes;
    h->zc = c.cols;
    h->zl_tune_us = c.us;
    h->zl_tuned = true;
}

// The batched Z-LAP mapping for tile size m without measuring (nothing is
// allocated): this process's or the cache file's choice, else the smallest
// lane group that holds m.
int known_batch_lanes(int device, int m)
{
    const std::string key = tune_key(device, "bzlap", m);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second.lanes;
    const char *path = std::getenv("QAP_TUNE_CACHE");
    if (path && *path) {
        const auto file = read_tune_file(path);
        const auto fit = file.find(key);
        if (fit != file.end()) return fit->second.lanes;
    }
    return m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64;
}

// Batched Z-LAP kernel for a batch whose largest tile is m: a lane count of
// k_bzlap, -1 for k_bzlap_s or -2 for k_bzlap_s2.  real, real_tiles: as for
// measure_bzlap (used only when the choice for m is not known yet).
int tuned_batch_lanes(int device, hipStream_t stream, int m, const double *real = nullptr, long long real_tiles = 0)
{
    return tuned_choice(tune_key(device, "bzlap", m), [&] { return measure_bzlap(stream, m, real, real_tiles); })
        .lanes;
}

}  // namespace
