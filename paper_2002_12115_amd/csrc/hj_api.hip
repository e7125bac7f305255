// hj_api.hip -- libhj runtime: device layout, resident solve loop, HIP graphs,
// batch descriptors, autotuner, and the C ABI declared in include/hj.h.
//
// Transfer policy (paper sections 3.2 and 3.3): every array is uploaded once
// and stays resident; a call to hj_sweep runs all its iterations on the
// device (as one HIP graph launch when use_graph is set) and brings back
// only the FP64 gosa values, 8 bytes per iteration. p and wrk2 are a
// ping-pong pair swapped by pointer, so there is no copy-back kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <mutex>
#include <shared_mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "hj_ga.hpp"
#include "hj_launch.hpp"

using namespace hj;

namespace {

constexpr uint64_t kSolverMagic = 0x686a736f6c766572ULL;  // "hjsolver"
constexpr uint64_t kBatchMagic = 0x686a626174636821ULL;   // "hjbatch!"
constexpr int kInputMask = (1 << 13) - 1;

thread_local std::string g_err;
thread_local double g_last_ms = 0.0;

int set_err(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct HipFail {
    hipError_t e;
    const char* expr;
    int line;
};

#define HIPCHK(x)                                              \
    do {                                                       \
        hipError_t e_ = (x);                                   \
        if (e_ != hipSuccess) throw HipFail{e_, #x, __LINE__}; \
    } while (0)

// Run an ABI body, mapping C++ failures to status codes.
template <typename F>
int guarded(F&& f)
{
    try {
        return f();
    } catch (const HipFail& h) {
        // clear the runtime's last error, so a later, unrelated launch check
        // does not report this one again (non-sticky errors such as OOM)
        (void)hipGetLastError();
        const int code = (h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation) ? HJ_ERR_OOM : HJ_ERR_HIP;
        return set_err(code, "%s failed at hj_api.hip:%d: %s (%s)", h.expr, h.line,
                       hipGetErrorName(h.e), hipGetErrorString(h.e));
    } catch (const std::bad_alloc&) {
        return set_err(HJ_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(HJ_ERR_ARG, "exception: %s", e.what());
    } catch (...) {
        return set_err(HJ_ERR_ARG, "unknown exception");
    }
}

// ---- layout -----------------------------------------------------------------

// Field q of a solve lives at slab + q*field_stride. Inside it, element
// (i,j,k) is at element offset (A-1) + i*S + j*P + k, where A = 128 bytes /
// element size: every row's k = 1 starts on a 128-byte line, P is a multiple
// of A and leaves room after k = nz-1 for the widest vector over-read. The
// field stride carries a 2304-byte stagger (9 * 256 B) so the 14 streams of a
// sweep start at different offsets modulo the DRAM interleave.
struct Layout {
    int nx = 0, ny = 0, nz = 0, esz = 0, A = 0;
    long long P = 0, S = 0;
    size_t field_bytes = 0, field_stride = 0, slab_bytes = 0;
    // A solve's slab (and each batch instance's part of a batch slab) also
    // holds the side array of the 64-cell-row tiles (side_index) after its fields.
    size_t fields_bytes = 0, side_bytes = 0;
    int side_kt = 0;
};

size_t stagger_bytes()
{
    static size_t s = [] {
        const char* e = getenv("HJ_STAGGER");
        long v = e ? atol(e) : 2304;
        if (v < 0) v = 0;
        return (size_t)((v + 255) / 256 * 256);
    }();
    return s;
}

bool make_layout(int dtype, int nx, int ny, int nz, Layout& L)
{
    if (nx < 3 || ny < 3 || nz < 3) return false;
    if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 24)) return false;
    L.nx = nx; L.ny = ny; L.nz = nz;
    L.esz = dtype == HJ_F64 ? 8 : 4;
    L.A = 128 / L.esz;
    L.P = pitch_of(L.esz, nz);
    L.S = (long long)ny * L.P;
    const long double bytes = (long double)nx * L.S * L.esz;
    if (bytes > (long double)(1ULL << 46)) return false;
    L.field_bytes = (size_t)nx * (size_t)L.S * (size_t)L.esz;
    L.field_stride = (L.field_bytes + 65535) / 65536 * 65536 + stagger_bytes();
    L.fields_bytes = (size_t)HJ_NFIELDS * L.field_stride;
    L.side_kt = kt64(nz);
    L.side_bytes = ((size_t)NCOEF * nx * L.side_kt * ny * 2 * L.esz + 255) / 256 * 256;
    L.slab_bytes = L.fields_bytes + L.side_bytes;
    return true;
}

// Refresh coefficient field's block of a side array (see side_index) from
// the field at `origin` (its element (0,0,0)); waits for the gather.
void gather_side(int dtype, const Layout& L, int field, const char* origin, char* side, hipStream_t st)
{
    const size_t blk = (size_t)L.nx * L.side_kt * L.ny * 2 * (field - HJ_A0);
    if (dtype == HJ_F64)
        HIPCHK(launch_side_gather<double>(reinterpret_cast<const double*>(origin),
                                          reinterpret_cast<double*>(side) + blk, L.nx, L.ny, L.nz, L.P, L.S, st));
    else
        HIPCHK(launch_side_gather<float>(reinterpret_cast<const float*>(origin), reinterpret_cast<float*>(side) + blk,
                                         L.nx, L.ny, L.nz, L.P, L.S, st));
    HIPCHK(hipStreamSynchronize(st));
}

int check_dtype(int dtype)
{
    if (dtype != HJ_F64 && dtype != HJ_F32) return set_err(HJ_ERR_DTYPE, "dtype %d is not HJ_F64 or HJ_F32", dtype);
    return HJ_OK;
}

// The one-iteration configuration: the base of the tuner's candidates and
// of gene decoding, and the kernel that runs the odd remainder iteration
// and the residual of two-iteration solves (non-temporal streams, 16-byte
// lanes, short i chunks: the best measured one-iteration family on MI355X).
hj_config default_config(int dtype)
{
    hj_config c;
    c.kernel = HJ_KERNEL_MARCH;
    c.bj = dtype == HJ_F64 ? 4 : 8;
    c.vec = dtype == HJ_F64 ? 2 : 4;
    c.ichunk = 4;
    c.nontemporal = 1;
    c.use_graph = 1;
    c.xcd_remap = 0;
    c.persistent = 0;
    c.tsteps = 1;
    c.reread = 0;
    return c;
}

bool same_config(const hj_config& a, const hj_config& b) { return memcmp(&a, &b, sizeof a) == 0; }

// The i-chunk that gives a grid about `target` workgroups under config c.
int ichunk_for(const hj_config& c, int nx, int ny, int nz, long long target)
{
    hj_config u = c;
    u.ichunk = 1;
    const TileCounts one = tile_counts(u, nx, ny, nz);
    const long long base = std::max<long long>(1, (long long)one.kt_n * one.jt_n);
    const long long nchunks = std::max<long long>(1, (target + base - 1) / base);
    return (int)std::max<long long>(1, (nx - 2 + nchunks - 1) / nchunks);
}

// The longest i-chunk that keeps the grid within max_wg workgroups (whole
// waves of resident workgroups leave no CU idle in a last, partial wave).
int ichunk_within(const hj_config& c, int nx, int ny, int nz, long long max_wg)
{
    hj_config u = c;
    u.ichunk = 1;
    const TileCounts one = tile_counts(u, nx, ny, nz);
    const long long base = std::max<long long>(1, (long long)one.kt_n * one.jt_n);
    const long long nchunks = std::max<long long>(1, max_wg / base);
    return (int)std::max<long long>(1, (nx - 2 + nchunks - 1) / nchunks);
}

// Reference configuration of the autotuner's parity gate: the plainest kernel.
hj_config reference_config(int dtype)
{
    hj_config c = default_config(dtype);
    c.kernel = HJ_KERNEL_DIRECT;
    c.bj = 4;
    c.vec = 1;
    c.nontemporal = 0;
    c.xcd_remap = 0;
    return c;
}

// ---- runtime calls that must not overlap a graph capture ----------------------
//
// A HIP graph capture on one thread is invalidated by a runtime call on any
// thread that allocates, frees or creates/destroys streams and graphs. The
// library's own such calls take this lock exclusively; captures take it
// shared, so captures may overlap each other but never those calls.
std::shared_mutex g_capture_mu;
using RuntimeLock = std::unique_lock<std::shared_mutex>;

void dev_alloc(void** p, size_t n)
{
    RuntimeLock lk(g_capture_mu);
    HIPCHK(hipMalloc(p, n));
}
void dev_free(void* p)
{
    RuntimeLock lk(g_capture_mu);
    (void)hipFree(p);
}
void host_alloc(void** p, size_t n)
{
    RuntimeLock lk(g_capture_mu);
    HIPCHK(hipHostMalloc(p, n, hipHostMallocDefault));
}
void host_free(void* p)
{
    RuntimeLock lk(g_capture_mu);
    (void)hipHostFree(p);
}
void stream_create(hipStream_t* s)
{
    RuntimeLock lk(g_capture_mu);
    HIPCHK(hipStreamCreateWithFlags(s, hipStreamNonBlocking));
}
void stream_destroy(hipStream_t s)
{
    RuntimeLock lk(g_capture_mu);
    (void)hipStreamDestroy(s);
}
void exec_destroy(hipGraphExec_t g)
{
    RuntimeLock lk(g_capture_mu);
    (void)hipGraphExecDestroy(g);
}

// Errors that mean a capture was disturbed from outside (another thread's
// runtime call); the work can still run eagerly.
bool capture_disturbed(hipError_t e)
{
    return e == hipErrorStreamCaptureInvalidated || e == hipErrorStreamCaptureImplicit ||
           e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureIsolation ||
           e == hipErrorStreamCaptureMerge || e == hipErrorStreamCaptureUnjoined ||
           e == hipErrorStreamCaptureUnmatched || e == hipErrorStreamCaptureWrongThread ||
           e == hipErrorCapturedEvent;
}

// ---- device buffers -----------------------------------------------------------

// A buffer the library allocates on demand and frees when its owner goes
// away (or at release()). Move-only: exactly one owner frees it.
template <void (*Alloc)(void**, size_t), void (*Free)(void*)>
struct OwnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    OwnedBuf() = default;
    OwnedBuf(const OwnedBuf&) = delete;
    OwnedBuf& operator=(const OwnedBuf&) = delete;
    OwnedBuf(OwnedBuf&& o) noexcept : p(o.p), bytes(o.bytes)
    {
        o.p = nullptr;
        o.bytes = 0;
    }
    OwnedBuf& operator=(OwnedBuf&& o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~OwnedBuf() { release(); }
    void ensure(size_t need)
    {
        if (need <= bytes) return;
        release();
        Alloc(&p, need);
        bytes = need;
    }
    void release()
    {
        if (p) Free(p);
        p = nullptr;
        bytes = 0;
    }
};

using DevBuf = OwnedBuf<dev_alloc, dev_free>;   // device memory
using PinBuf = OwnedBuf<host_alloc, host_free>; // pinned host memory

struct GraphEntry {
    int n_iter;
    uint64_t omega_bits;
    int parity;
    hj_config cfg;
    double* out;
    hipGraphExec_t exec;
};

uint64_t bits_of(double x)
{
    uint64_t u;
    memcpy(&u, &x, 8);
    return u;
}

// Iterations whose per-tile gosa partials are kept before a finalize.
int chunk_iters(int n_iter, long long tiles)
{
    long long ch = std::min<long long>(256, n_iter);
    const long long cap = (32LL << 20) / std::max<long long>(1, tiles);  // <= 256 MiB of partials
    ch = std::max<long long>(1, std::min(ch, cap));
    return (int)ch;
}

// The executable graphs of a handle's recent loops (at most 8, oldest
// evicted first). Graphs are launched on the handle's stream `st`; before
// an exec is destroyed, that stream is drained, so no launch of it can
// still be queued or running. (A stream under capture by the caller has run
// nothing yet: it is not drained.)
struct GraphCache {
    std::vector<GraphEntry> v;
    hipStream_t st = nullptr;
    hipGraphExec_t find(int n, double omega, int parity, const hj_config& c, double* out)
    {
        for (auto& e : v)
            if (e.n_iter == n && e.omega_bits == bits_of(omega) && e.parity == parity &&
                same_config(e.cfg, c) && e.out == out)
                return e.exec;
        return nullptr;
    }
    void drain()
    {
        if (!st) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
            (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
    }
    void add(const GraphEntry& e)
    {
        if (v.size() >= 8) {
            drain();
            exec_destroy(v.front().exec);
            v.erase(v.begin());
        }
        v.push_back(e);
    }
    void clear()
    {
        if (v.empty()) return;
        drain();
        for (auto& e : v) exec_destroy(e.exec);
        v.clear();
    }
};

template <typename Enq>
hipGraphExec_t capture(hipStream_t cap, Enq&& enqueue)
{
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
        enqueue(cap);
    } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(cap, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
    }
    HIPCHK(hipStreamEndCapture(cap, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    return exec;
}

// The graph of an n_iter loop from parity `parity`: from the cache, or
// captured and cached. nullptr when the capture was disturbed from outside
// (the caller then enqueues the same work eagerly; nothing ran on the device).
template <typename Enq>
hipGraphExec_t find_or_capture(GraphCache& graphs, hipStream_t cap, int n_iter, double omega, int parity,
                               const hj_config& cfg, double* out, Enq&& enqueue)
{
    if (hipGraphExec_t ex = graphs.find(n_iter, omega, parity, cfg, out)) return ex;
    hipGraphExec_t ex = nullptr;
    try {
        ex = capture(cap, [&](hipStream_t s) { enqueue(parity, s); });
    } catch (const HipFail& f) {
        if (!capture_disturbed(f.e)) throw;
        (void)hipGetLastError();
        return nullptr;
    }
    graphs.add(GraphEntry{n_iter, bits_of(omega), parity, cfg, out, ex});
    return ex;
}

std::mutex g_reg_mu;
std::set<void*> g_registry;

void reg_add(void* h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_registry.insert(h);
}
bool reg_has(void* h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return g_registry.count(h) != 0;
}
void reg_del(void* h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_registry.erase(h);
}

// Optional record of every autotuner measurement (HJ_TUNE_LOG=<csv path>).
void tune_log(const char* what, int dtype, int nx, int ny, int nz, const hj_config& c, double ms,
              const char* verdict)
{
    const char* path = getenv("HJ_TUNE_LOG");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s,%s,%d,%d,%d,%d,%d,%d,%d,%d,%d,%d,%.6f,%s,%d,%d\n", what, dtype == HJ_F64 ? "f64" : "f32", nx,
            ny, nz, c.kernel, c.bj, c.vec, c.ichunk, c.nontemporal, c.xcd_remap, c.persistent, ms, verdict, c.tsteps,
            c.reread);
    fclose(f);
}

int median_index_sort(std::vector<float>& t)
{
    std::sort(t.begin(), t.end());
    return (int)(t.size() / 2);
}

// ---- tuning cache ------------------------------------------------------------
//
// With HJ_TUNE_CACHE=<path>, every successful autotune records its winner as
// one text line, and a new handle whose (kind, GPU architecture, dtype,
// shape key) matches a line starts from that configuration:
//   <kind> <arch> <f64|f32> <key> <kernel> <bj> <vec> <ichunk> <nt> <remap> <persistent> <ms> <tsteps> <reread>
std::mutex g_cache_mu;

const char* cache_path()
{
    const char* p = getenv("HJ_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

std::string device_arch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a.resize(c);
    return a.empty() ? "unknown" : a;
}

std::string solve_key(int nx, int ny, int nz)
{
    char b[64];
    snprintf(b, sizeof b, "%dx%dx%d", nx, ny, nz);
    return b;
}

std::string batch_key(const std::vector<Layout>& L)
{
    uint64_t h = 1469598103934665603ULL;  // FNV-1a over the instance shapes
    for (const Layout& l : L)
        for (int d : {l.nx, l.ny, l.nz}) {
            h ^= (uint64_t)(uint32_t)d;
            h *= 1099511628211ULL;
        }
    char b[64];
    snprintf(b, sizeof b, "n%zu-%016llx", L.size(), (unsigned long long)h);
    return b;
}

bool cache_get(const char* kind, int dtype, const std::string& key, hj_config& c)
{
    const char* path = cache_path();
    if (!path) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE* f = fopen(path, "r");
    if (!f) return false;
    const std::string arch = device_arch();
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[32], a[64], d[8], kk[128];
        hj_config x = default_config(dtype);
        double ms = 0;
        const int got = sscanf(line, "%31s %63s %7s %127s %d %d %d %d %d %d %d %lf %d %d", k, a, d, kk, &x.kernel,
                               &x.bj, &x.vec, &x.ichunk, &x.nontemporal, &x.xcd_remap, &x.persistent, &ms,
                               &x.tsteps, &x.reread);
        if (got < 12) continue;
        if (got < 13) x.tsteps = 1;
        if (got < 14) x.reread = 0;
        if (strcmp(k, kind) || arch != a || strcmp(d, dtype == HJ_F64 ? "f64" : "f32") || key != kk) continue;
        c = x;
        found = true;  // the last matching line wins
    }
    fclose(f);
    return found;
}

void cache_put(const char* kind, int dtype, const std::string& key, const hj_config& c, double ms)
{
    const char* path = cache_path();
    if (!path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    const std::string arch = device_arch();
    const char* d = dtype == HJ_F64 ? "f64" : "f32";
    std::vector<std::string> keep;
    if (FILE* f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof line, f)) {
            char k[32], a[64], dd[8], kk[128];
            if (sscanf(line, "%31s %63s %7s %127s", k, a, dd, kk) == 4 && !strcmp(k, kind) && arch == a &&
                !strcmp(dd, d) && key == kk)
                continue;  // replaced below
            keep.emplace_back(line);
        }
        fclose(f);
    }
    FILE* f = fopen(path, "w");
    if (!f) return;
    for (const std::string& l : keep) fputs(l.c_str(), f);
    fprintf(f, "%s %s %s %s %d %d %d %d %d %d %d %.6f %d %d\n", kind, arch.c_str(), d, key.c_str(), c.kernel,
            c.bj, c.vec, c.ichunk, c.nontemporal, c.xcd_remap, c.persistent, ms, c.tsteps, c.reread);
    fclose(f);
}

// ---- autotuner measurement --------------------------------------------------

// What the autotuner needs from a solve or a batch.
struct TuneOps {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::function<void(const hj_config&)> set;     // select a configuration (may throw)
    std::function<void()> restore;                 // back to the saved state
    std::function<void(int)> run;                  // enqueue n sweeps
    // the device regions the parity gate compares (the current p of each grid)
    std::function<std::vector<std::pair<const void*, size_t>>()> result;
};

// Host-side failure injection for the tuner's error paths (no kernel is
// changed and nothing faults): HJ_TUNE_INJECT holds rules separated by ';',
// each "launch:<field>=<v>,..." or "parity:<field>=<v>,...", with fields named
// as in hj_config. A candidate matching every field of a launch rule is
// scored as if it had failed to launch (it is not run); one matching a parity
// rule is run and then scored as if its field differed from the reference's.
enum class Inject { none, launch, parity };

Inject injected_failure(const hj_config& c)
{
    const char* env = getenv("HJ_TUNE_INJECT");
    if (!env || !*env) return Inject::none;
    const std::pair<const char*, int> fields[] = {
        {"kernel", c.kernel},       {"bj", c.bj},           {"vec", c.vec},
        {"ichunk", c.ichunk},       {"nontemporal", c.nontemporal}, {"use_graph", c.use_graph},
        {"xcd_remap", c.xcd_remap}, {"persistent", c.persistent},   {"tsteps", c.tsteps},
        {"reread", c.reread}};
    std::string all(env);
    size_t pos = 0;
    while (pos <= all.size()) {
        size_t end = all.find(';', pos);
        if (end == std::string::npos) end = all.size();
        const std::string rule = all.substr(pos, end - pos);
        pos = end + 1;
        const size_t colon = rule.find(':');
        if (colon == std::string::npos) continue;
        const std::string mode = rule.substr(0, colon);
        if (mode != "launch" && mode != "parity") continue;
        bool match = true, any = false;
        size_t q = colon + 1;
        while (q < rule.size() && match) {
            size_t e = rule.find(',', q);
            if (e == std::string::npos) e = rule.size();
            const std::string kv = rule.substr(q, e - q);
            q = e + 1;
            const size_t eq = kv.find('=');
            if (eq == std::string::npos) { match = false; break; }
            const std::string name = kv.substr(0, eq);
            const int val = atoi(kv.c_str() + eq + 1);
            bool known = false;
            for (const auto& f : fields)
                if (name == f.first) {
                    known = true;
                    match = match && f.second == val;
                }
            match = match && known;
            any = true;
        }
        if (match && any) return mode == "launch" ? Inject::launch : Inject::parity;
    }
    return Inject::none;
}

// Times configurations on the caller's arrays. The first configuration
// evaluated is the reference; every later one must leave a result bitwise
// equal to it after the same sweeps, or it scores as failed (INFINITY).
struct Evaluator {
    TuneOps ops;
    int n_sweeps = 1, repeats = 1;
    const char* kind = "solve";
    int dtype = HJ_F64, nx = 0, ny = 0, nz = 0;
    DevBuf ref, cnt;
    bool have_ref = false;

    double eval(const hj_config& c)
    {
        const Inject inj = injected_failure(c);
        if (inj == Inject::launch) {
            tune_log(kind, dtype, nx, ny, nz, c, INFINITY, "launch-failed");
            return INFINITY;
        }
        try {
            ops.set(c);
            ops.restore();
            ops.run(n_sweeps);
        } catch (const HipFail&) {
            (void)hipGetLastError();
            tune_log(kind, dtype, nx, ny, nz, c, INFINITY, "launch-failed");
            return INFINITY;  // a candidate that does not launch is never chosen
        }
        if (inj == Inject::parity) {
            HIPCHK(hipStreamSynchronize(ops.st));
            tune_log(kind, dtype, nx, ny, nz, c, INFINITY, "parity-failed");
            return INFINITY;
        }
        const std::vector<std::pair<const void*, size_t>> res = ops.result();
        if (!have_ref) {
            size_t total = 0;
            for (const auto& r : res) total += r.second;
            ref.ensure(total);
            size_t o = 0;
            for (const auto& r : res) {
                HIPCHK(hipMemcpyAsync(static_cast<char*>(ref.p) + o, r.first, r.second, hipMemcpyDeviceToDevice,
                                      ops.st));
                o += r.second;
            }
            have_ref = true;
        } else {
            unsigned long long bad = 0;
            cnt.ensure(8);
            HIPCHK(hipMemcpyAsync(cnt.p, &bad, 8, hipMemcpyHostToDevice, ops.st));
            size_t o = 0;
            for (const auto& r : res) {
                HIPCHK(launch_diff(r.first, static_cast<const char*>(ref.p) + o, r.second,
                                   static_cast<unsigned long long*>(cnt.p), ops.st));
                o += r.second;
            }
            HIPCHK(hipMemcpyAsync(&bad, cnt.p, 8, hipMemcpyDeviceToHost, ops.st));
            HIPCHK(hipStreamSynchronize(ops.st));
            if (bad) {
                tune_log(kind, dtype, nx, ny, nz, c, INFINITY, "parity-failed");
                return INFINITY;
            }
        }
        std::vector<float> t;
        for (int r = 0; r < repeats; ++r) {
            HIPCHK(hipEventRecord(ops.e0, ops.st));
            ops.run(n_sweeps);
            HIPCHK(hipEventRecord(ops.e1, ops.st));
            HIPCHK(hipEventSynchronize(ops.e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ops.e0, ops.e1));
            t.push_back(ms);
        }
        const double med = t[median_index_sort(t)];
        tune_log(kind, dtype, nx, ny, nz, c, med, "ok");
        return med;
    }
};

// ---- the genetic search's gene ------------------------------------------------
//
// 11 bits, every value naming a configuration (codes that do not apply to a
// mode are ignored, unusable ones fold onto usable ones):
//   bit 0      kernel: 0 direct, 1 march; with bit 10: 0 flat, 1 march with
//              two iterations per pass (batches: 0 flat, 1 march, with bit
//              10 two iterations per pass)
//   bits 1-2   bj: 1, 2, 4, 8 (direct: 1 reads as 2; two-iteration: 14, 6, 4, 8)
//   bits 3-4   vec (march, one iteration): FP64 1, 2, 1, 2; FP32 1, 2, 4, 4;
//              two-iteration passes: bit 3 is reread, bit 4 the row layout:
//              single solves 64-cell rows with a halo wave (vec 2, where bj
//              14 reads as 12), batches two 30-cell rows per wave (vec 4,
//              bj codes 14, 6, 22, 30)
//   bits 5-7   one of 8 i-chunk lengths (march kernels)
//   bit 8      non-temporal streams
//   bit 9      XCD renumbering (single solves, two-iteration batches) /
//              persistent grid (one-iteration batches)
//   bit 10     see bit 0
// A flat kernel that does not fit the grid reads as the march kernel.
constexpr int kGeneBits = 11;

// The 8 i-chunk lengths a gene can name for one grid: the chunk that gives
// about 512, 1024, ..., 65536 workgroups; for two-iteration passes, whose
// chunks recompute their halo planes and whose workgroups are few and long,
// the longest chunk within 256, 512, 768, 1024, 2048, 4096, 8192 or 24576
// workgroups (whole waves on a chip of 256 CUs).
// The gene (paper sections 4 and 5.1.2: one bit per decision, every value
// measured) over this kernel's configurations. Every gene names a
// configuration that the exhaustive search also measures (its candidate list
// includes every decoded gene), and two-iteration genes carry the settings
// the exhaustive search keeps for those passes (temporal loads, XCD
// renumbering), so both searches cover the same space.
//  bit 10: two iterations per pass (1) or one (0).
//  two iterations: bit 0 the row layout (set: 64-cell rows with a halo wave
//    for single solves, two 30-cell rows per wave for batches; clear: 62-cell
//    rows); bits 1-2 bj (62-cell rows 4, 6, 8, 14; 64-cell rows 4, 6, 8, 12;
//    30-cell rows 6, 14, 22, 30); bit 3 reread; bits 5-7 the i-chunk (single
//    solves: the longest within 256, 512, 768, 1024, 1536, 2048, 4096 or 16384
//    workgroups; batches 8, 12, 16, 24, 32, 48, 64 or 128 planes); bits 4, 8
//    and 9 unused.
//  one iteration: bit 0 the march kernel (set), else for single solves the
//    flat kernel (bit 3 set) or the direct kernel, for batches the flat
//    kernel; bits 1-2 bj 1, 2, 4, 8 (flat and direct read 1 as 2); bits 3-4
//    vec of the march kernel 1, 2, 1, 2 (FP64) or 1, 2, 4, 4 (FP32); bits 5-6
//    the i-chunk (single solves: about 1024, 2048, 4096 or 8192 workgroups;
//    batches 2, 4, 8 or 16 planes); bit 7 unused; bit 8 nontemporal; bit 9
//    xcd_remap of the march kernel (single solves) or the persistent grid
//    (batches).
bool decode_gene(uint32_t g, int dtype, int nx, int ny, int nz, bool batch, hj_config& c)
{
    static const int kBj[4] = {1, 2, 4, 8};
    static const int kBj62[4] = {4, 6, 8, 14}, kBj64[4] = {4, 6, 8, 12}, kBj30[4] = {6, 14, 22, 30};
    static const int kVec64[4] = {1, 2, 1, 2}, kVec32[4] = {1, 2, 4, 4};
    static const long long kTwoWg[8] = {256, 512, 768, 1024, 1536, 2048, 4096, 16384};
    static const int kTwoPlanes[8] = {8, 12, 16, 24, 32, 48, 64, 128};
    c = default_config(dtype);
    const int b0 = g & 1, bi = (g >> 1) & 3, b3 = (g >> 3) & 1, vi = (g >> 3) & 3;
    const int sel3 = (g >> 5) & 7, sel2 = (g >> 5) & 3;
    c.use_graph = 1;
    c.persistent = 0;
    c.reread = 0;
    if ((g >> 10) & 1) {
        c.kernel = HJ_KERNEL_MARCH;
        c.tsteps = 2;
        c.nontemporal = 0;
        c.xcd_remap = 1;
        c.reread = b3;
        if (!b0) {
            c.vec = 1;
            c.bj = kBj62[bi];
        } else if (batch) {
            c.vec = 4;
            c.bj = kBj30[bi];
        } else {
            c.vec = 2;
            c.bj = kBj64[bi];
        }
        c.ichunk = batch ? kTwoPlanes[sel3] : ichunk_within(c, nx, ny, nz, kTwoWg[sel3]);
        return config_supported(dtype, c);
    }
    c.tsteps = 1;
    c.nontemporal = (g >> 8) & 1;
    const int b9 = (g >> 9) & 1;
    c.bj = kBj[bi];
    c.vec = dtype == HJ_F64 ? kVec64[vi] : kVec32[vi];
    c.xcd_remap = 0;
    if (b0) {
        c.kernel = HJ_KERNEL_MARCH;
        if (batch) c.persistent = b9;
        else c.xcd_remap = b9;
        c.ichunk = batch ? (2 << sel2) : ichunk_for(c, nx, ny, nz, 1024LL << sel2);
    } else {
        c.kernel = (batch || b3) ? HJ_KERNEL_FLAT : HJ_KERNEL_DIRECT;
        if (c.bj == 1) c.bj = 2;
        c.vec = 1;
        if (c.kernel == HJ_KERNEL_DIRECT) {
            c.ichunk = 1;
        } else {
            if (batch) c.persistent = b9;
            c.ichunk = batch ? (2 << sel2) : ichunk_for(c, nx, ny, nz, 1024LL << sel2);
            if (!batch && !config_fits(dtype, c, nx, ny, nz)) {
                c.kernel = HJ_KERNEL_MARCH;           // a run too wide for the grid: the march kernel
                c.ichunk = ichunk_for(c, nx, ny, nz, 1024LL << sel2);
            }
        }
    }
    return config_supported(dtype, c);
}

}  // namespace

// ---- partials of the allocation-free sweep ------------------------------------

// Per-tile gosa partials of hj_sweep_noalloc: a file-scope device array, one
// copy on every GPU the library runs on, held until the process ends. Host
// code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
static __device__ __align__(256) double scratch[HJ_NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev`, which must be the current
// device; looked up at the first call for that device.
double* scratch_on(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) throw HipFail{hipErrorInvalidDevice, "scratch_on(dev)", __LINE__};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

// ============================================================================
// single solve
// ============================================================================

struct hj_solver_s {
    uint64_t magic = kSolverMagic;
    int dtype = HJ_F64;
    int device = 0;           // the device current at creation
    Layout L;
    char* slab = nullptr;
    bool owns_slab = false;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    hipStream_t cap = nullptr;
    int parity = 0;           // 0: field HJ_P holds the current p, 1: field HJ_WRK2 does
    unsigned uploaded = 0;
    hj_config cfg;
    DevBuf part, gosa;
    PinBuf host_gosa;
    GraphCache graphs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // hj_snapshot: a dense device copy of p, sent to the host on a stream of its own
    DevBuf snap;
    hipStream_t xfer = nullptr;
    hipEvent_t snap_ready = nullptr, snap_sent = nullptr;
    bool snap_pending = false;

    char* field(int q) const { return slab + (size_t)q * L.field_stride; }
    // element (0,0,0) of field q
    char* origin(int q) const { return field(q) + (size_t)(L.A - 1) * L.esz; }
    char* side() const { return slab + L.fields_bytes; }

    template <typename T>
    Grid<T> grid(int par) const
    {
        Grid<T> g;
        for (int q = 0; q < NCOEF; ++q) g.coef[q] = reinterpret_cast<const T*>(origin(HJ_A0 + q));
        g.src = reinterpret_cast<const T*>(origin(par ? HJ_WRK2 : HJ_P));
        g.dst = reinterpret_cast<T*>(origin(par ? HJ_P : HJ_WRK2));
        g.nx = L.nx; g.ny = L.ny; g.nz = L.nz; g.P = L.P; g.S = L.S;
        g.side = reinterpret_cast<const T*>(side());
        g.side_kt = L.side_kt;
        return g;
    }

    // The single-iteration configuration: cfg itself, or, for two-iteration
    // passes, the one that runs an odd remainder and the residual.
    hj_config single_cfg() const
    {
        if (!fused_of(cfg)) return cfg;
        hj_config c = default_config(dtype);
        c.ichunk = ichunk_for(c, L.nx, L.ny, L.nz, 4096);
        c.nontemporal = cfg.nontemporal;
        c.use_graph = cfg.use_graph;
        return c;
    }
    long long tiles_of(const hj_config& c) const { return tile_counts(c, L.nx, L.ny, L.nz).tiles(); }
    // the runtime queries of cfg's launches, made now (outside any capture)
    void prime() const
    {
        if (dtype == HJ_F64) prime_remap<double>(cfg);
        else prime_remap<float>(cfg);
    }
    // Partials per iteration slot (room for either kernel's tiles).
    long long stride() const { return std::max(tiles_of(cfg), tiles_of(single_cfg())); }
    long long tiles() const { return tiles_of(cfg); }
    // Iterations per block of partials; pairs of a two-iteration pass never straddle two blocks.
    int chunk_of(int n_iter) const
    {
        int ch = chunk_iters(std::max(n_iter, 1), stride());
        if (fused_of(cfg)) ch = std::max(2, ch & ~1);
        return ch;
    }
    int launches(int n_iter) const { return fused_of(cfg) ? n_iter / 2 + (n_iter & 1) : n_iter; }

    hipError_t launch_one(const hj_config& c, int par, double omega, bool write, double* part_out,
                          hipStream_t st) const
    {
        if (dtype == HJ_F64) return launch_sweep<double>(c, grid<double>(par), omega, write, part_out, st);
        return launch_sweep<float>(c, grid<float>(par), (float)omega, write, part_out, st);
    }
    hipError_t launch_two(int par, double omega, double* p1, double* p2, hipStream_t st) const
    {
        if (dtype == HJ_F64) return launch_fused<double>(cfg, grid<double>(par), omega, p1, p2, st);
        return launch_fused<float>(cfg, grid<float>(par), (float)omega, p1, p2, st);
    }

    // Enqueue n_iter iterations starting from parity `par`, gosa history to
    // out. The per-tile partials of up to `ch` iterations (0: chunk_of) at a
    // time go to pt (null: the handle's buffer), stride() doubles per
    // iteration. Returns the parity after them (one flip per launch).
    int enqueue(int n_iter, double omega, int par, double* out, hipStream_t st, double* pt = nullptr,
                int ch = 0) const
    {
        const bool two = fused_of(cfg);
        const hj_config one = single_cfg();
        const long long sd = stride();
        if (ch <= 0) ch = chunk_of(n_iter);
        if (!pt) pt = static_cast<double*>(part.p);
        for (int it0 = 0; it0 < n_iter;) {
            const int n_here = std::min(ch, n_iter - it0);
            int slot = 0;
            if (two) {
                for (; slot + 1 < n_here; slot += 2) {
                    HIPCHK(launch_two(par, omega, pt + slot * sd, pt + (slot + 1) * sd, st));
                    par ^= 1;
                }
                if (slot > 0)
                    HIPCHK(launch_finalize(pt, sd, (int)tiles_of(cfg), nullptr, 1, slot, out + it0, st));
            }
            if (slot < n_here) {
                const int first = slot;
                const hj_config& c = two ? one : cfg;
                for (; slot < n_here; ++slot) {
                    HIPCHK(launch_one(c, par, omega, true, pt + slot * sd, st));
                    par ^= 1;
                }
                HIPCHK(launch_finalize(pt + first * sd, sd, (int)tiles_of(c), nullptr, 1, slot - first,
                                       out + it0 + first, st));
            }
            it0 += n_here;
        }
        return par;
    }

    void reserve(int n_iter)
    {
        const size_t need_part = (size_t)chunk_of(n_iter) * (size_t)stride() * 8;
        const size_t need_gosa = (size_t)std::max(n_iter, 1) * 8;
        if (need_part > part.bytes || need_gosa > gosa.bytes) {
            graphs.clear();  // graphs hold the old addresses
            part.ensure(need_part);
            gosa.ensure(need_gosa);
        }
    }

    // Enqueue the whole loop on `stream`, as a graph replay when configured.
    void run(int n_iter, double omega, double* out)
    {
        hipGraphExec_t ex = cfg.use_graph ? find_or_capture(graphs, cap, n_iter, omega, parity, cfg, out,
                                                            [&](int par, hipStream_t s) {
                                                                enqueue(n_iter, omega, par, out, s);
                                                            })
                                          : nullptr;
        if (ex) {
            HIPCHK(hipGraphLaunch(ex, stream));
            parity ^= (launches(n_iter) & 1);
        } else {
            parity = enqueue(n_iter, omega, parity, out, stream);
        }
    }
};

namespace {

int check_solver(hj_solver h)
{
    if (!h || !reg_has(h) || h->magic != kSolverMagic)
        return set_err(HJ_ERR_HANDLE, "invalid or destroyed hj_solver handle");
    return HJ_OK;
}

int solver_init(hj_solver* out, int dtype, int nx, int ny, int nz, void* dev_slab,
                unsigned long long slab_bytes, void* stream)
{
    if (!out) return set_err(HJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (int rc = check_dtype(dtype)) return rc;
    Layout L;
    if (!make_layout(dtype, nx, ny, nz, L))
        return set_err(HJ_ERR_SHAPE, "shape %dx%dx%d is invalid (each >= 3, within limits)", nx, ny, nz);
    if (dev_slab) {
        if (slab_bytes < L.slab_bytes)
            return set_err(HJ_ERR_ARG, "slab of %llu bytes is smaller than the %zu needed", slab_bytes, L.slab_bytes);
        if (reinterpret_cast<uintptr_t>(dev_slab) % 256)
            return set_err(HJ_ERR_ARG, "device slab must be 256-byte aligned");
    }
    hj_solver h = new hj_solver_s();
    h->dtype = dtype;
    h->L = L;
    h->cfg = default_config(dtype);
    try {
        HIPCHK(hipGetDevice(&h->device));
        (void)scratch_on(h->device);  // set-up of hj_sweep_noalloc on this device
        if (dev_slab) {
            h->slab = static_cast<char*>(dev_slab);
        } else {
            dev_alloc(reinterpret_cast<void**>(&h->slab), L.slab_bytes);
            h->owns_slab = true;
        }
        if (stream) {
            h->stream = static_cast<hipStream_t>(stream);
        } else {
            stream_create(&h->stream);
            h->owns_stream = true;
        }
        stream_create(&h->cap);
        HIPCHK(hipEventCreate(&h->ev0));
        HIPCHK(hipEventCreate(&h->ev1));
        h->graphs.st = h->stream;
    } catch (...) {
        if (h->owns_slab && h->slab) dev_free(h->slab);
        if (h->owns_stream && h->stream) stream_destroy(h->stream);
        if (h->cap) stream_destroy(h->cap);
        if (h->ev0) (void)hipEventDestroy(h->ev0);
        if (h->ev1) (void)hipEventDestroy(h->ev1);
        delete h;
        throw;
    }
    reg_add(h);
    *out = h;
    return HJ_OK;
}

// Host <-> device copies of one dense field. They go through two pinned
// staging buffers shared by the process, so the PCIe transfer of one chunk of
// rows overlaps the host-side copy (or FP64 -> FP32 rounding) of the next.
// Rows too long for a staging buffer, and host arrays that are pinned
// already, take a direct pitched copy.
struct Stager {
    static constexpr size_t kBytes = 32u << 20;
    std::mutex mu;
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    void ensure()
    {
        for (int q = 0; q < 2; ++q) {
            if (!buf[q]) host_alloc(&buf[q], kBytes);
            if (!ev[q]) HIPCHK(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming));
        }
    }
};

Stager& stager()
{
    static Stager* s = new Stager();  // lives until the process ends
    return *s;
}

// Runs f(begin, end) over [0, n) split across up to 8 host threads (one
// thread copies pageable memory at about 10 GB/s, well under the PCIe link).
template <typename F>
void host_parallel(size_t n, size_t min_per_thread, F f)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t t = std::min<size_t>({8, hw, std::max<size_t>(1, n / min_per_thread)});
    if (t < 2) {
        f(size_t(0), n);
        return;
    }
    const size_t per = (n + t - 1) / t;
    std::vector<std::thread> th;
    th.reserve(t - 1);
    for (size_t i = 1; i < t && i * per < n; ++i) th.emplace_back(f, i * per, std::min(n, (i + 1) * per));
    f(size_t(0), std::min(n, per));
    for (std::thread& x : th) x.join();
}

void par_memcpy(void* dst, const void* src, size_t bytes)
{
    host_parallel(bytes, size_t(4) << 20, [=](size_t b, size_t e) {
        memcpy(static_cast<char*>(dst) + b, static_cast<const char*>(src) + b, e - b);
    });
}

void round_rows(float* dst, const double* src, size_t n)
{
    host_parallel(n, size_t(1) << 20, [=](size_t b, size_t e) {
        for (size_t q = b; q < e; ++q) dst[q] = (float)src[q];  // round to nearest even
    });
}

// What a host-side array argument points to: ordinary (pageable) memory;
// pinned host memory (hipHostMalloc, or a torch pin_memory tensor), which a
// DMA copy reads or writes directly with no staging; or device memory,
// which is not a host array.
enum class HostMem { pageable, pinned, device };

HostMem host_mem(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory is not an error here
        return HostMem::pageable;
    }
    if (a.type == hipMemoryTypeHost) return HostMem::pinned;
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeArray) return HostMem::device;
    return HostMem::pageable;  // managed memory: reachable from the host
}

bool host_pinned(const void* p) { return host_mem(p) == HostMem::pinned; }

// src holds nx*ny rows of nz values: doubles when src_f64, else the field's type.
void copy_in(const Layout& L, char* field, const void* src, bool src_f64, hipStream_t st)
{
    char* dst = field + (size_t)(L.A - 1) * L.esz;
    const size_t row = (size_t)L.nz * L.esz, pitch = (size_t)L.P * L.esz;
    const size_t rows = (size_t)L.nx * L.ny;
    const bool convert = src_f64 && L.esz == 4;
    if (row > Stager::kBytes || (!convert && host_pinned(src))) {
        std::vector<float> tmp;
        const void* s = src;
        if (convert) {
            tmp.resize(rows * L.nz);
            round_rows(tmp.data(), static_cast<const double*>(src), tmp.size());
            s = tmp.data();
        }
        HIPCHK(hipMemcpy2DAsync(dst, pitch, s, row, row, rows, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return;
    }
    Stager& sg = stager();
    std::lock_guard<std::mutex> lk(sg.mu);
    sg.ensure();
    const size_t chunk = Stager::kBytes / row;
    bool used[2] = {false, false};
    int b = 0;
    for (size_t r0 = 0; r0 < rows; r0 += chunk, b ^= 1) {
        const size_t n = std::min(chunk, rows - r0);
        if (used[b]) HIPCHK(hipEventSynchronize(sg.ev[b]));
        if (convert)
            round_rows(static_cast<float*>(sg.buf[b]), static_cast<const double*>(src) + r0 * L.nz, n * L.nz);
        else
            par_memcpy(sg.buf[b], static_cast<const char*>(src) + r0 * row, n * row);
        HIPCHK(hipMemcpy2DAsync(dst + r0 * pitch, pitch, sg.buf[b], row, row, n, hipMemcpyHostToDevice, st));
        HIPCHK(hipEventRecord(sg.ev[b], st));
        used[b] = true;
    }
    HIPCHK(hipStreamSynchronize(st));
}

void copy_out(const Layout& L, const char* field, void* dst, hipStream_t st)
{
    const char* src = field + (size_t)(L.A - 1) * L.esz;
    const size_t row = (size_t)L.nz * L.esz, pitch = (size_t)L.P * L.esz;
    const size_t rows = (size_t)L.nx * L.ny;
    if (row > Stager::kBytes || host_pinned(dst)) {
        HIPCHK(hipMemcpy2DAsync(dst, row, src, pitch, row, rows, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return;
    }
    Stager& sg = stager();
    std::lock_guard<std::mutex> lk(sg.mu);
    sg.ensure();
    const size_t chunk = Stager::kBytes / row;
    size_t prev_r0 = 0, prev_n = 0;
    int b = 0;
    for (size_t r0 = 0; r0 < rows; r0 += chunk, b ^= 1) {
        const size_t n = std::min(chunk, rows - r0);
        HIPCHK(hipMemcpy2DAsync(sg.buf[b], row, src + r0 * pitch, pitch, row, n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(sg.ev[b], st));
        if (prev_n) {  // drain the other buffer while this chunk is in flight
            HIPCHK(hipEventSynchronize(sg.ev[b ^ 1]));
            par_memcpy(static_cast<char*>(dst) + prev_r0 * row, sg.buf[b ^ 1], prev_n * row);
        }
        prev_r0 = r0;
        prev_n = n;
    }
    if (prev_n) {
        HIPCHK(hipEventSynchronize(sg.ev[b ^ 1]));
        par_memcpy(static_cast<char*>(dst) + prev_r0 * row, sg.buf[b ^ 1], prev_n * row);
    }
    HIPCHK(hipStreamSynchronize(st));
}

int validate_config(int dtype, const hj_config* c)
{
    if (!c) return set_err(HJ_ERR_ARG, "config is NULL");
    if (!config_supported(dtype, *c))
        return set_err(HJ_ERR_ARG, "unsupported config kernel=%d bj=%d vec=%d ichunk=%d for dtype %d",
                       c->kernel, c->bj, c->vec, c->ichunk, dtype);
    return HJ_OK;
}

// The autotuner's candidates for one grid; cus is the device's CU count
// (two-iteration chunks are sized to whole waves of resident workgroups).
// Every configuration a gene names (decode_gene), added to a candidate list,
// so that the exhaustive search covers the genetic search's space.
void add_gene_space(std::vector<hj_config>& out, int dtype, int nx, int ny, int nz, bool batch)
{
    for (uint32_t g = 0; g < (1u << kGeneBits); ++g) {
        hj_config x;
        if (!decode_gene(g, dtype, nx, ny, nz, batch, x)) continue;
        if (!batch && !config_fits(dtype, x, nx, ny, nz)) continue;
        bool dup = false;
        for (const hj_config& y : out) dup = dup || same_config(x, y);
        if (!dup) out.push_back(x);
    }
}

std::vector<hj_config> candidates(int dtype, int nx, int ny, int nz, bool batch, int cus)
{
    std::vector<hj_config> out;
    const hj_config base = default_config(dtype);
    if (!batch) {
        for (int bj : {2, 4, 8})
            for (int nt : {0, 1}) {
                hj_config c = base;
                c.kernel = HJ_KERNEL_DIRECT;
                c.bj = bj;
                c.vec = 1;
                c.nontemporal = nt;
                c.xcd_remap = 0;
                out.push_back(c);
            }
    }
    const int ni = nx - 2;
    std::vector<int> vecs = dtype == HJ_F64 ? std::vector<int>{1, 2} : std::vector<int>{1, 2, 4};
    for (int bj : {1, 2, 4, 8})
        for (int v : vecs) {
            const long long kt = (nz - 2 + 64 * v - 1) / (64 * v);
            const long long jt = (ny - 2 + bj - 1) / bj;
            const long long base_tiles = kt * jt;
            std::vector<int> ich;
            for (long long target : {1024LL, 2048LL, 4096LL, 8192LL, 16384LL}) {
                long long nchunks = (target + base_tiles - 1) / base_tiles;
                int c = (int)std::max<long long>(1, (ni + nchunks - 1) / nchunks);
                c = std::min(c, std::max(ni, 1));
                if (std::find(ich.begin(), ich.end(), c) == ich.end()) ich.push_back(c);
            }
            for (int c : ich)
                for (int nt : {0, 1})
                    for (int rm : {0, 1}) {
                        hj_config x = base;
                        x.kernel = HJ_KERNEL_MARCH;
                        x.bj = bj;
                        x.vec = v;
                        x.ichunk = c;
                        x.nontemporal = nt;
                        x.xcd_remap = batch ? 0 : rm;
                        x.persistent = batch ? rm : 0;
                        if (config_supported(dtype, x)) out.push_back(x);
                    }
        }
    if (!batch) {
        // flat runs of consecutive (j,k) cells
        for (int nw : {2, 4, 8})
            for (int target : {1024, 2048, 4096, 8192})
                for (int nt : {0, 1}) {
                    hj_config x = base;
                    x.kernel = HJ_KERNEL_FLAT;
                    x.bj = nw;
                    x.vec = 1;
                    x.nontemporal = nt;
                    x.xcd_remap = 0;
                    x.ichunk = ichunk_for(x, nx, ny, nz, target);
                    bool dup = false;
                    for (const hj_config& y : out) dup = dup || same_config(x, y);
                    if (!dup && config_fits(dtype, x, nx, ny, nz)) out.push_back(x);
                }
        // two iterations per pass (62-cell rows, or 64-cell rows with a halo
        // wave): long chunks (the halo planes of a chunk are recomputed), sized
        // to 1 .. 64 waves of resident workgroups; XCD renumbering lets
        // neighbouring tiles share their halo reads in L2
        static const std::pair<int, int> kFusedShapes[] = {{1, 6},  {1, 8},  {1, 14}, {2, 4},  {2, 6},
                                                           {2, 8},  {2, 12}, {4, 14}, {4, 30}};
        for (const auto& vb : kFusedShapes)
            for (int rr : {0, 1})
                for (int rm : {1}) {
                    hj_config x = base;
                    x.kernel = HJ_KERNEL_MARCH;
                    x.bj = vb.second;
                    x.vec = vb.first;
                    x.tsteps = 2;
                    x.reread = rr;
                    x.nontemporal = 0;
                    x.xcd_remap = rm;
                    if (!config_supported(dtype, x)) continue;
                    const int occ = dtype == HJ_F64 ? fused_occupancy<double>(x) : fused_occupancy<float>(x);
                    const long long cap = (long long)std::max(occ, 1) * std::max(cus, 1);
                    for (int m : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64}) {
                        x.ichunk = ichunk_within(x, nx, ny, nz, m * cap);
                        bool dup = false;
                        for (const hj_config& y : out) dup = dup || same_config(x, y);
                        if (!dup) out.push_back(x);
                    }
                }
    }
    add_gene_space(out, dtype, nx, ny, nz, batch);
    return out;
}

// A default i-chunk that gives the grid a few thousand workgroups.
int default_ichunk(int dtype, const hj_config& c, int nx, int ny, int nz)
{
    const long long kt = (nz - 2 + 64 * c.vec - 1) / (64 * c.vec);
    const long long jt = (ny - 2 + c.bj - 1) / c.bj;
    const long long target = 4096;
    const long long nchunks = std::max<long long>(1, (target + kt * jt - 1) / (kt * jt));
    (void)dtype;
    return (int)std::max<long long>(1, (nx - 2 + nchunks - 1) / nchunks);
}

// Starting configuration of a new single solve before any tuning: two
// iterations per pass on 64-cell rows with a halo wave (8 rows per tile,
// coefficients kept in registers, XCD-aware tile numbering), in the longest
// i-chunk that keeps the grid to one wave of resident workgroups. Of this
// family it is the measured best on the 128^2x256 and 256^2x512 interiors and
// within 5% of the best on 512^2x1024. Falls back to the one-iteration kernel
// when the grid or the device query rules it out.
hj_config start_config(int dtype, int nx, int ny, int nz)
{
    hj_config c = default_config(dtype);
    c.kernel = HJ_KERNEL_MARCH;
    c.bj = 8;
    c.vec = 2;
    c.tsteps = 2;
    c.reread = 0;
    c.nontemporal = 0;
    c.xcd_remap = 1;
    int dev = 0, cus = 0;
    const int occ = dtype == HJ_F64 ? fused_occupancy<double>(c) : fused_occupancy<float>(c);
    if (occ > 0 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
        c.ichunk = ichunk_within(c, nx, ny, nz, (long long)occ * cus);
        if (config_fits(dtype, c, nx, ny, nz)) return c;
    }
    (void)hipGetLastError();
    c = default_config(dtype);
    c.ichunk = default_ichunk(dtype, c, nx, ny, nz);
    return c;
}

// Starting configuration, or the tuning cache's entry for this problem.
void apply_start_config(hj_solver h)
{
    h->cfg = start_config(h->dtype, h->L.nx, h->L.ny, h->L.nz);
    hj_config c;
    if (cache_get("solve", h->dtype, solve_key(h->L.nx, h->L.ny, h->L.nz), c) &&
        config_fits(h->dtype, c, h->L.nx, h->L.ny, h->L.nz)) {
        c.use_graph = 1;
        c.persistent = 0;
        h->cfg = c;
    }
    h->prime();
}

}  // namespace

extern "C" {

const char* hj_status_string(int s)
{
    switch (s) {
    case HJ_OK: return "HJ_OK";
    case HJ_ERR_ARG: return "HJ_ERR_ARG";
    case HJ_ERR_SHAPE: return "HJ_ERR_SHAPE";
    case HJ_ERR_DTYPE: return "HJ_ERR_DTYPE";
    case HJ_ERR_OOM: return "HJ_ERR_OOM";
    case HJ_ERR_HIP: return "HJ_ERR_HIP";
    case HJ_ERR_STATE: return "HJ_ERR_STATE";
    case HJ_ERR_HANDLE: return "HJ_ERR_HANDLE";
    case HJ_ERR_TUNE: return "HJ_ERR_TUNE";
    default: return "HJ_ERR_UNKNOWN";
    }
}

const char* hj_last_error(void) { return g_err.c_str(); }

double hj_last_sweep_ms(void) { return g_last_ms; }

int hj_slab_bytes(int dtype, int nx, int ny, int nz, unsigned long long* bytes)
{
    if (!bytes) return set_err(HJ_ERR_ARG, "bytes is NULL");
    if (int rc = check_dtype(dtype)) return rc;
    Layout L;
    if (!make_layout(dtype, nx, ny, nz, L)) return set_err(HJ_ERR_SHAPE, "invalid shape %dx%dx%d", nx, ny, nz);
    *bytes = L.slab_bytes;
    return HJ_OK;
}

int hj_create(hj_solver* out, int dtype, int nx, int ny, int nz, void* stream)
{
    return guarded([&]() -> int {
        const int rc = solver_init(out, dtype, nx, ny, nz, nullptr, 0, stream);
        if (rc == HJ_OK) apply_start_config(*out);
        return rc;
    });
}

int hj_attach(hj_solver* out, int dtype, int nx, int ny, int nz, void* device_slab,
              unsigned long long slab_bytes, void* stream)
{
    if (!device_slab) return set_err(HJ_ERR_ARG, "device_slab is NULL");
    return guarded([&]() -> int {
        const int rc = solver_init(out, dtype, nx, ny, nz, device_slab, slab_bytes, stream);
        if (rc == HJ_OK) apply_start_config(*out);
        return rc;
    });
}

namespace {

int solver_upload(hj_solver h, int field, const void* src, bool src_f64)
{
    if (int rc = check_solver(h)) return rc;
    if (!src) return set_err(HJ_ERR_ARG, "host_src is NULL");
    if (host_mem(src) == HostMem::device) return set_err(HJ_ERR_ARG, "host_src is device memory, not a host array");
    if (field == HJ_WRK2) return set_err(HJ_ERR_ARG, "HJ_WRK2 is derived from HJ_P and cannot be uploaded");
    if (field < 0 || field >= HJ_WRK2) return set_err(HJ_ERR_ARG, "field %d out of range", field);
    return guarded([&]() -> int {
        if (field == HJ_P) {
            copy_in(h->L, h->field(HJ_P), src, src_f64, h->stream);
            copy_in(h->L, h->field(HJ_WRK2), src, src_f64, h->stream);
            h->parity = 0;
        } else {
            copy_in(h->L, h->field(field), src, src_f64, h->stream);
            gather_side(h->dtype, h->L, field, h->origin(field), h->side(), h->stream);
        }
        h->uploaded |= 1u << field;
        return HJ_OK;
    });
}

}  // namespace

int hj_upload(hj_solver h, int field, const void* src) { return solver_upload(h, field, src, false); }

int hj_upload_f64(hj_solver h, int field, const double* src) { return solver_upload(h, field, src, true); }

int hj_download(hj_solver h, int field, void* dst)
{
    if (int rc = check_solver(h)) return rc;
    if (!dst) return set_err(HJ_ERR_ARG, "host_dst is NULL");
    if (host_mem(dst) == HostMem::device) return set_err(HJ_ERR_ARG, "host_dst is device memory, not a host array");
    if (field < 0 || field >= HJ_NFIELDS) return set_err(HJ_ERR_ARG, "field %d out of range", field);
    return guarded([&]() -> int {
        int q = field;
        if (field == HJ_P || field == HJ_WRK2) q = h->parity ? HJ_WRK2 : HJ_P;
        copy_out(h->L, h->field(q), dst, h->stream);
        return HJ_OK;
    });
}

int hj_snapshot(hj_solver h, void* host_dst)
{
    if (int rc = check_solver(h)) return rc;
    if (!host_dst) return set_err(HJ_ERR_ARG, "host_dst is NULL");
    if (host_mem(host_dst) == HostMem::device)
        return set_err(HJ_ERR_ARG, "host_dst is device memory, not a host array");
    return guarded([&]() -> int {
        const Layout& L = h->L;
        const size_t row = (size_t)L.nz * L.esz, pitch = (size_t)L.P * L.esz, rows = (size_t)L.nx * L.ny;
        // each resource is made once; a failure part way leaves the rest to the next call
        if (!h->snap_ready) HIPCHK(hipEventCreateWithFlags(&h->snap_ready, hipEventDisableTiming));
        if (!h->snap_sent) HIPCHK(hipEventCreateWithFlags(&h->snap_sent, hipEventDisableTiming));
        if (!h->xfer) stream_create(&h->xfer);
        h->snap.ensure(rows * row);
        // the previous snapshot's transfer must have read the buffer first
        if (h->snap_pending) HIPCHK(hipStreamWaitEvent(h->stream, h->snap_sent, 0));
        // the field, made dense on the device (fast), then one flat copy over
        // PCIe (a pitched host copy of short rows runs well below the link)
        const char* cur = h->field(h->parity ? HJ_WRK2 : HJ_P) + (size_t)(L.A - 1) * L.esz;
        HIPCHK(hipMemcpy2DAsync(h->snap.p, row, cur, pitch, row, rows, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipEventRecord(h->snap_ready, h->stream));
        HIPCHK(hipStreamWaitEvent(h->xfer, h->snap_ready, 0));
        HIPCHK(hipMemcpyAsync(host_dst, h->snap.p, rows * row, hipMemcpyDeviceToHost, h->xfer));
        HIPCHK(hipEventRecord(h->snap_sent, h->xfer));
        h->snap_pending = true;
        return HJ_OK;
    });
}

int hj_snapshot_wait(hj_solver h)
{
    if (int rc = check_solver(h)) return rc;
    return guarded([&]() -> int {
        if (h->snap_pending) HIPCHK(hipEventSynchronize(h->snap_sent));
        h->snap_pending = false;
        return HJ_OK;
    });
}

int hj_sweep(hj_solver h, int n_iter, double omega, double* gosa_last, double* gosa_hist)
{
    if (int rc = check_solver(h)) return rc;
    if (n_iter < 0) return set_err(HJ_ERR_ARG, "n_iter %d < 0", n_iter);
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded (mask 0x%x)", h->uploaded);
    if (n_iter == 0) return HJ_OK;
    return guarded([&]() -> int {
        h->reserve(n_iter);
        double* out = static_cast<double*>(h->gosa.p);
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        h->run(n_iter, omega, out);
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        h->host_gosa.ensure((size_t)n_iter * 8);
        HIPCHK(hipMemcpyAsync(h->host_gosa.p, out, (size_t)n_iter * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        g_last_ms = ms;
        const double* hg = static_cast<const double*>(h->host_gosa.p);
        if (gosa_hist) memcpy(gosa_hist, hg, (size_t)n_iter * 8);
        if (gosa_last) *gosa_last = hg[n_iter - 1];
        return HJ_OK;
    });
}

int hj_sweep_async(hj_solver h, int n_iter, double omega, double* dev_gosa_hist)
{
    if (int rc = check_solver(h)) return rc;
    if (n_iter < 0) return set_err(HJ_ERR_ARG, "n_iter %d < 0", n_iter);
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded (mask 0x%x)", h->uploaded);
    if (n_iter == 0) return HJ_OK;
    return guarded([&]() -> int {
        h->reserve(n_iter);
        double* out = dev_gosa_hist ? dev_gosa_hist : static_cast<double*>(h->gosa.p);
        h->run(n_iter, omega, out);
        return HJ_OK;
    });
}

int hj_sweep_noalloc(hj_solver h, int n_iter, double omega, double* dev_gosa_hist)
{
    if (int rc = check_solver(h)) return rc;
    if (n_iter < 0) return set_err(HJ_ERR_ARG, "n_iter %d < 0", n_iter);
    if (!dev_gosa_hist) return set_err(HJ_ERR_ARG, "dev_gosa_hist is NULL");
    const long long sd = h->stride();
    const bool two = fused_of(h->cfg);
    const long long fit = (long long)HJ_NOALLOC_SCRATCH_DOUBLES / sd;  // iterations of partials that fit
    if (fit < (two ? 2 : 1))
        return set_err(HJ_ERR_ARG, "%lld gosa partials per iteration (%s) exceed the %d-double scratch of "
                       "hj_sweep_noalloc", sd, two ? "two-iteration passes" : "one-iteration passes",
                       HJ_NOALLOC_SCRATCH_DOUBLES);
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded (mask 0x%x)", h->uploaded);
    if (n_iter == 0) return HJ_OK;
    return guarded([&]() -> int {
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != h->device)
            return set_err(HJ_ERR_ARG, "current device %d is not the handle's device %d", dev, h->device);
        int ch = h->chunk_of(n_iter);
        if (ch > fit) ch = two ? (int)(fit & ~1LL) : (int)fit;
        // eager launches on the handle's stream: no graph is instantiated
        h->parity = h->enqueue(n_iter, omega, h->parity, dev_gosa_hist, h->stream, scratch_on(dev), ch);
        return HJ_OK;
    });
}

int hj_residual(hj_solver h, double* gosa)
{
    if (int rc = check_solver(h)) return rc;
    if (!gosa) return set_err(HJ_ERR_ARG, "gosa is NULL");
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded (mask 0x%x)", h->uploaded);
    return guarded([&]() -> int {
        h->reserve(1);
        double* pt = static_cast<double*>(h->part.p);
        double* out = static_cast<double*>(h->gosa.p);
        const hj_config one = h->single_cfg();
        const long long nt = h->tiles_of(one);
        HIPCHK(h->launch_one(one, h->parity, 0.0, false, pt, h->stream));
        HIPCHK(launch_finalize(pt, nt, (int)nt, nullptr, 1, 1, out, h->stream));
        h->host_gosa.ensure(8);
        HIPCHK(hipMemcpyAsync(h->host_gosa.p, out, 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        *gosa = *static_cast<const double*>(h->host_gosa.p);
        return HJ_OK;
    });
}

int hj_get_config(hj_solver h, hj_config* out)
{
    if (int rc = check_solver(h)) return rc;
    if (!out) return set_err(HJ_ERR_ARG, "out is NULL");
    *out = h->cfg;
    return HJ_OK;
}

int hj_set_config(hj_solver h, const hj_config* cfg)
{
    if (int rc = check_solver(h)) return rc;
    if (int rc = validate_config(h->dtype, cfg)) return rc;
    if (!config_fits(h->dtype, *cfg, h->L.nx, h->L.ny, h->L.nz))
        return set_err(HJ_ERR_ARG, "the flat kernel with bj %d does not fit a %dx%dx%d grid", cfg->bj, h->L.nx,
                       h->L.ny, h->L.nz);
    return guarded([&]() -> int {
        h->graphs.clear();
        h->cfg = *cfg;
        h->cfg.persistent = 0;
        if (h->cfg.tsteps == 0) h->cfg.tsteps = 1;
        if (h->cfg.tsteps == 1) h->cfg.reread = 0;
        h->prime();
        return HJ_OK;
    });
}

namespace {

// Tuning operations over a single solve: the saved state is the current
// field, restored into both halves of the ping-pong pair. The saved copy and
// the evaluator's buffers are freed with the session. If the session ends
// without finish() (an exception), the field and configuration are put back.
struct SolverTuning {
    hj_solver h;
    DevBuf save;
    Evaluator ev;
    hj_config keep;
    bool saved = false, finished = false;

    SolverTuning(const SolverTuning&) = delete;
    SolverTuning& operator=(const SolverTuning&) = delete;
    ~SolverTuning()
    {
        if (finished) return;
        try {
            if (saved) restore();
            (void)hipStreamSynchronize(h->stream);
            h->graphs.clear();
        } catch (...) {
        }
        (void)hipGetLastError();
        h->cfg = keep;
    }

    SolverTuning(hj_solver hh, int n_sweeps, int repeats) : h(hh)
    {
        const Layout& L = h->L;
        keep = h->cfg;
        save.ensure(L.field_bytes);
        HIPCHK(hipMemcpyAsync(save.p, h->field(h->parity ? HJ_WRK2 : HJ_P), L.field_bytes,
                              hipMemcpyDeviceToDevice, h->stream));
        saved = true;
        ev.n_sweeps = n_sweeps;
        ev.repeats = repeats;
        ev.kind = "solve";
        ev.dtype = h->dtype;
        ev.nx = L.nx; ev.ny = L.ny; ev.nz = L.nz;
        ev.ops.st = h->stream;
        ev.ops.e0 = h->ev0;
        ev.ops.e1 = h->ev1;
        ev.ops.set = [this](const hj_config& c) {
            if (!config_fits(h->dtype, c, h->L.nx, h->L.ny, h->L.nz))
                throw HipFail{hipErrorInvalidValue, "flat kernel does not fit", __LINE__};
            h->graphs.clear();
            h->cfg = c;
            h->cfg.use_graph = 0;
            h->reserve(ev.n_sweeps);
        };
        ev.ops.restore = [this] { restore(); };
        ev.ops.run = [this](int n) { h->run(n, 0.8, static_cast<double*>(h->gosa.p)); };
        ev.ops.result = [this] {
            return std::vector<std::pair<const void*, size_t>>{
                {(const void*)h->field(h->parity ? HJ_WRK2 : HJ_P), h->L.field_bytes}};
        };
    }
    void restore()
    {
        HIPCHK(hipMemcpyAsync(h->field(HJ_P), save.p, h->L.field_bytes, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->field(HJ_WRK2), save.p, h->L.field_bytes, hipMemcpyDeviceToDevice, h->stream));
        h->parity = 0;
    }
    // Put the state back and install the winner (or the old configuration).
    int finish(const hj_config& win, double win_ms, hj_config* best, double* best_ms)
    {
        restore();
        HIPCHK(hipStreamSynchronize(h->stream));
        h->graphs.clear();
        finished = true;
        if (!std::isfinite(win_ms)) {
            h->cfg = keep;
            return set_err(HJ_ERR_TUNE, "no candidate configuration passed");
        }
        h->cfg = win;
        h->cfg.use_graph = keep.use_graph;
        h->prime();
        cache_put("solve", h->dtype, solve_key(h->L.nx, h->L.ny, h->L.nz), h->cfg, win_ms);
        if (best) *best = h->cfg;
        if (best_ms) *best_ms = win_ms;
        return HJ_OK;
    }
};

int solver_tunable(hj_solver h, int n_sweeps, int repeats)
{
    if (int rc = check_solver(h)) return rc;
    if (n_sweeps < 1 || repeats < 1) return set_err(HJ_ERR_ARG, "n_sweeps and repeats must be >= 1");
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded");
    return HJ_OK;
}

}  // namespace

int hj_autotune(hj_solver h, int n_sweeps, int repeats, hj_config* best, double* best_ms)
{
    if (int rc = solver_tunable(h, n_sweeps, repeats)) return rc;
    return guarded([&]() -> int {
        SolverTuning tu(h, n_sweeps, repeats);
        tu.ev.eval(reference_config(h->dtype));  // the parity reference (also a contender below)
        hj_config win = tu.keep;
        double win_ms = INFINITY;
        int dev = 0, cus = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        for (const hj_config& c : candidates(h->dtype, h->L.nx, h->L.ny, h->L.nz, false, cus)) {
            const double ms = tu.ev.eval(c);
            if (ms < win_ms) {
                win_ms = ms;
                win = c;
            }
        }
        return tu.finish(win, win_ms, best, best_ms);
    });
}

int hj_autotune_ga(hj_solver h, int population, int generations, unsigned long long seed, double pc,
                   double pm, int n_sweeps, int repeats, hj_config* best, double* best_ms, int* evaluations)
{
    if (int rc = solver_tunable(h, n_sweeps, repeats)) return rc;
    if (population < 1 || generations < 1 || !(pc >= 0.0 && pc <= 1.0) || !(pm >= 0.0 && pm <= 1.0))
        return set_err(HJ_ERR_ARG, "need population, generations >= 1 and 0 <= pc, pm <= 1");
    return guarded([&]() -> int {
        SolverTuning tu(h, n_sweeps, repeats);
        tu.ev.eval(reference_config(h->dtype));
        const Layout& L = h->L;
        std::vector<std::pair<hj_config, double>> seen;  // one measurement per configuration
        auto time_of = [&](uint32_t g) -> double {
            hj_config c;
            if (!decode_gene(g, h->dtype, L.nx, L.ny, L.nz, false, c)) return hjga::kFailTime;
            for (auto& e : seen)
                if (same_config(e.first, c)) return e.second;
            const double ms = tu.ev.eval(c);
            const double t = std::isfinite(ms) ? ms * 1e-3 : hjga::kFailTime;
            seen.emplace_back(c, t);
            return t;
        };
        const hjga::Result r = hjga::run(kGeneBits, population, generations, seed, pc, pm, time_of);
        hj_config win = tu.keep;
        double win_ms = INFINITY;
        if (r.best_time < hjga::kFailTime && decode_gene(r.best_gene, h->dtype, L.nx, L.ny, L.nz, false, win))
            win_ms = r.best_time * 1e3;
        if (evaluations) *evaluations = r.evaluations;
        return tu.finish(win, win_ms, best, best_ms);
    });
}

int hj_sync(hj_solver h)
{
    if (int rc = check_solver(h)) return rc;
    return guarded([&]() -> int {
        HIPCHK(hipStreamSynchronize(h->stream));
        return HJ_OK;
    });
}

int hj_get_stream(hj_solver h, void** stream)
{
    if (int rc = check_solver(h)) return rc;
    if (!stream) return set_err(HJ_ERR_ARG, "stream is NULL");
    *stream = h->stream;
    return HJ_OK;
}

int hj_destroy(hj_solver h)
{
    if (int rc = check_solver(h)) return rc;
    reg_del(h);
    (void)hipStreamSynchronize(h->stream);
    if (h->xfer) {
        (void)hipStreamSynchronize(h->xfer);
        stream_destroy(h->xfer);
    }
    if (h->snap_ready) (void)hipEventDestroy(h->snap_ready);
    if (h->snap_sent) (void)hipEventDestroy(h->snap_sent);
    h->snap.release();
    h->graphs.clear();
    h->part.release();
    h->gosa.release();
    h->host_gosa.release();
    if (h->owns_slab) dev_free(h->slab);
    if (h->owns_stream) stream_destroy(h->stream);
    stream_destroy(h->cap);
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    h->magic = 0;
    delete h;
    return HJ_OK;
}

int hj_stream_probe(hj_solver h, int vec, int ichunk, int n_rep, double* ms)
{
    if (int rc = check_solver(h)) return rc;
    if (n_rep < 1 || !ms) return set_err(HJ_ERR_ARG, "need n_rep >= 1 and ms");
    if ((h->uploaded & kInputMask) != (unsigned)kInputMask)
        return set_err(HJ_ERR_STATE, "not every input field is uploaded");
    return guarded([&]() -> int {
        // writes the interior of the ping-pong partner, which the next sweep
        // overwrites before reading it: the solve's state is unchanged
        auto go = [&](hipStream_t st) -> hipError_t {
            if (h->dtype == HJ_F64) return launch_stream_probe<double>(h->grid<double>(h->parity), vec, ichunk, st);
            return launch_stream_probe<float>(h->grid<float>(h->parity), vec, ichunk, st);
        };
        HIPCHK(go(h->stream));
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        for (int r = 0; r < n_rep; ++r) HIPCHK(go(h->stream));
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        HIPCHK(hipEventSynchronize(h->ev1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, h->ev0, h->ev1));
        *ms = t / n_rep;
        return HJ_OK;
    });
}

int hj_copy_probe(void* dst, const void* src, unsigned long long bytes, void* stream, double* ms)
{
    if (!dst || !src) return set_err(HJ_ERR_ARG, "null buffer");
    if (bytes % 16) return set_err(HJ_ERR_ARG, "bytes must be a multiple of 16");
    return guarded([&]() -> int {
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        HIPCHK(hipEventRecord(a, st));
        hipError_t e = launch_copy(dst, src, bytes, st);
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        HIPCHK(e);
        if (ms) *ms = t;
        return HJ_OK;
    });
}

}  // extern "C"

// ============================================================================
// batch of independent solves
// ============================================================================

namespace {

// Default batch configuration: the march kernel, one iteration per pass.
hj_config batch_default(int dtype)
{
    hj_config c = default_config(dtype);
    c.kernel = HJ_KERNEL_MARCH;
    c.bj = 4;
    c.vec = 1;
    c.ichunk = 16;
    c.xcd_remap = 0;
    c.persistent = 0;
    return c;
}

}  // namespace

// The flattened tile list of every instance of a batch for one configuration.
struct BatchTiles {
    DevBuf d_inst, d_tile_inst, d_seg;
    int ntiles = 0, grid = 0;

    void release()
    {
        d_inst.release();
        d_tile_inst.release();
        d_seg.release();
    }
};

struct hj_batch_s {
    uint64_t magic = kBatchMagic;
    int dtype = HJ_F32;
    int n = 0;
    std::vector<Layout> L;
    std::vector<size_t> off;       // byte offset of each instance in the slab
    char* slab = nullptr;
    size_t slab_bytes = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    hipStream_t cap = nullptr;
    int parity = 0;
    std::vector<unsigned> uploaded;
    hj_config cfg;
    int cus = 256;
    // tile lists of the current configuration and, for two-iteration passes,
    // of the one-iteration configuration that runs an odd remainder and the residual
    BatchTiles tl, tl1;
    hj_config tiled_for;
    bool tiled = false;
    DevBuf part, gosa;
    PinBuf host_gosa;
    GraphCache graphs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    char* field(int inst, int q) const { return slab + off[inst] + (size_t)q * L[inst].field_stride; }
    char* origin(int inst, int q) const { return field(inst, q) + (size_t)(L[inst].A - 1) * L[inst].esz; }
    char* side(int inst) const { return slab + off[inst] + L[inst].fields_bytes; }

    bool two() const { return fused_of(cfg); }
    hj_config single_cfg() const
    {
        if (!two()) return cfg;
        hj_config c = batch_default(dtype);
        c.nontemporal = 1;
        c.use_graph = cfg.use_graph;
        return c;
    }
    const BatchTiles& single_tiles() const { return two() ? tl1 : tl; }

    template <typename T>
    void build_tiles_t(const hj_config& c, BatchTiles& out)
    {
        std::vector<Instance<T>> inst(n);
        std::vector<int> tile_inst;
        std::vector<int> seg(n + 1, 0);
        for (int t = 0; t < n; ++t) {
            const Layout& l = L[t];
            Instance<T>& d = inst[t];
            d.f[0] = reinterpret_cast<T*>(origin(t, HJ_P));
            d.f[1] = reinterpret_cast<T*>(origin(t, HJ_WRK2));
            for (int q = 0; q < NCOEF; ++q) d.coef[q] = reinterpret_cast<const T*>(origin(t, HJ_A0 + q));
            d.nx = l.nx; d.ny = l.ny; d.nz = l.nz; d.P = l.P; d.S = l.S;
            d.side = reinterpret_cast<const T*>(side(t));
            d.side_kt = l.side_kt;
            const TileCounts tc = tile_counts(c, l.nx, l.ny, l.nz);
            d.kt_n = tc.kt_n;
            d.jt_n = tc.jt_n;
            d.ichunk = c.ichunk;
            d.tile0 = (int)tile_inst.size();
            seg[t] = d.tile0;
            const long long nt = tc.tiles();
            if (tile_inst.size() + nt > 0x7fffffffLL) throw std::bad_alloc();
            tile_inst.insert(tile_inst.end(), (size_t)nt, t);
        }
        seg[n] = (int)tile_inst.size();
        out.ntiles = (int)tile_inst.size();
        if (fused_of(c)) {
            // two-iteration lists: (instance, tile within it) pairs. Without
            // XCD renumbering the tiles with the most planes go first
            // (stable), so that the short remainder chunks fill the launch's
            // last round; with it the list stays instance-major, so that each
            // XCD's eighth of the list holds whole instances.
            std::vector<int> order(out.ntiles);
            std::vector<int> planes(out.ntiles);
            for (int i = 0; i < out.ntiles; ++i) {
                const Instance<T>& d = inst[tile_inst[i]];
                const int t = i - d.tile0, ic = t / (d.kt_n * d.jt_n), ib = 1 + ic * d.ichunk;
                planes[i] = std::min(ib + d.ichunk, d.nx - 1) - ib;
                order[i] = i;
            }
            if (!c.xcd_remap)
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return planes[a] > planes[b]; });
            std::vector<int> pairs(2 * (size_t)out.ntiles);
            for (int i = 0; i < out.ntiles; ++i) {
                const int at = order[i], ti = tile_inst[at];
                pairs[2 * (size_t)i] = ti;
                pairs[2 * (size_t)i + 1] = at - inst[ti].tile0;
            }
            tile_inst.swap(pairs);
        }
        out.d_inst.ensure(sizeof(Instance<T>) * std::max(n, 1));
        out.d_tile_inst.ensure(sizeof(int) * std::max(tile_inst.size(), (size_t)1));
        out.d_seg.ensure(sizeof(int) * (n + 1));
        // on the batch's own stream (a copy on the legacy stream would disturb
        // graph captures running on other threads)
        HIPCHK(hipMemcpyAsync(out.d_inst.p, inst.data(), sizeof(Instance<T>) * n, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(out.d_tile_inst.p, tile_inst.data(), sizeof(int) * tile_inst.size(),
                              hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(out.d_seg.p, seg.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (c.persistent) {
            const int occ = batch_occupancy<T>(c);
            out.grid = std::max(1, std::min(out.ntiles, std::max(occ, 1) * cus));
        } else {
            out.grid = out.ntiles;
        }
    }

    void build_list(const hj_config& c, BatchTiles& out)
    {
        if (dtype == HJ_F64) build_tiles_t<double>(c, out);
        else build_tiles_t<float>(c, out);
    }

    void build_tiles()
    {
        if (tiled && same_config(tiled_for, cfg)) return;
        for (const Layout& l : L)  // every launch comes through here: never run a kernel that does not fit
            if (!config_fits(dtype, cfg, l.nx, l.ny, l.nz))
                throw HipFail{hipErrorInvalidValue, "configuration does not fit an instance", __LINE__};
        graphs.clear();
        tiled = false;
        build_list(cfg, tl);
        if (two()) build_list(single_cfg(), tl1);
        tiled_for = cfg;
        tiled = true;
    }

    // Partials per iteration slot (room for either list's tiles).
    long long stride() const { return two() ? std::max(tl.ntiles, tl1.ntiles) : tl.ntiles; }
    // Iterations per block of partials; pairs of a two-iteration pass never straddle two blocks.
    int chunk_of(int n_iter) const
    {
        int ch = chunk_iters(std::max(n_iter, 1), stride());
        if (two()) ch = std::max(2, ch & ~1);
        return ch;
    }
    int launches(int n_iter) const { return two() ? n_iter / 2 + (n_iter & 1) : n_iter; }

    hipError_t launch_one(const hj_config& c, const BatchTiles& t, int par, double omega, bool write,
                          double* part_out, hipStream_t st) const
    {
        if (dtype == HJ_F64)
            return launch_batch<double>(c, static_cast<const Instance<double>*>(t.d_inst.p),
                                        static_cast<const int*>(t.d_tile_inst.p), t.ntiles, t.grid, par, omega,
                                        write, part_out, st);
        return launch_batch<float>(c, static_cast<const Instance<float>*>(t.d_inst.p),
                                   static_cast<const int*>(t.d_tile_inst.p), t.ntiles, t.grid, par, (float)omega,
                                   write, part_out, st);
    }
    hipError_t launch_two(int par, double omega, double* p1, double* p2, hipStream_t st) const
    {
        if (dtype == HJ_F64)
            return launch_batch_fused<double>(cfg, static_cast<const Instance<double>*>(tl.d_inst.p),
                                              static_cast<const int*>(tl.d_tile_inst.p), tl.ntiles, par, omega,
                                              p1, p2, st);
        return launch_batch_fused<float>(cfg, static_cast<const Instance<float>*>(tl.d_inst.p),
                                         static_cast<const int*>(tl.d_tile_inst.p), tl.ntiles, par, (float)omega,
                                         p1, p2, st);
    }
    hipError_t finalize(const double* pt, const BatchTiles& t, int slots, double* out, hipStream_t st) const
    {
        return launch_finalize(pt, stride(), t.ntiles, static_cast<const int*>(t.d_seg.p), n, slots, out, st);
    }

    // Enqueue n_iter iterations from parity `par`, gosa history [n_iter][n]
    // to out. Returns the parity after them (one flip per launch).
    int enqueue(int n_iter, double omega, int par, double* out, hipStream_t st) const
    {
        const long long sd = stride();
        const int ch = chunk_of(n_iter);
        const hj_config one = single_cfg();
        const BatchTiles& t1 = single_tiles();
        double* pt = static_cast<double*>(part.p);
        for (int it0 = 0; it0 < n_iter;) {
            const int n_here = std::min(ch, n_iter - it0);
            int slot = 0;
            if (two()) {
                for (; slot + 1 < n_here; slot += 2) {
                    HIPCHK(launch_two(par, omega, pt + slot * sd, pt + (slot + 1) * sd, st));
                    par ^= 1;
                }
                if (slot > 0) HIPCHK(finalize(pt, tl, slot, out + (long long)it0 * n, st));
            }
            if (slot < n_here) {
                const int first = slot;
                for (; slot < n_here; ++slot) {
                    HIPCHK(launch_one(one, t1, par, omega, true, pt + slot * sd, st));
                    par ^= 1;
                }
                HIPCHK(finalize(pt + first * sd, t1, slot - first, out + (long long)(it0 + first) * n, st));
            }
            it0 += n_here;
        }
        return par;
    }

    void reserve(int n_iter)
    {
        build_tiles();
        const size_t need_part = (size_t)chunk_of(n_iter) * (size_t)std::max<long long>(stride(), 1) * 8;
        const size_t need_gosa = (size_t)std::max(n_iter, 1) * (size_t)n * 8;
        if (need_part > part.bytes || need_gosa > gosa.bytes) {
            graphs.clear();
            part.ensure(need_part);
            gosa.ensure(need_gosa);
        }
    }

    void run(int n_iter, double omega, double* out)
    {
        hipGraphExec_t ex = cfg.use_graph ? find_or_capture(graphs, cap, n_iter, omega, parity, cfg, out,
                                                            [&](int par, hipStream_t s) {
                                                                enqueue(n_iter, omega, par, out, s);
                                                            })
                                          : nullptr;
        if (ex) {
            HIPCHK(hipGraphLaunch(ex, stream));
            parity ^= (launches(n_iter) & 1);
        } else {
            parity = enqueue(n_iter, omega, parity, out, stream);
        }
    }

    bool all_uploaded() const
    {
        for (unsigned u : uploaded)
            if ((u & kInputMask) != (unsigned)kInputMask) return false;
        return true;
    }
};

namespace {

bool batch_fits(const hj_batch_s* b, const hj_config& c)
{
    for (const Layout& l : b->L)
        if (!config_fits(b->dtype, c, l.nx, l.ny, l.nz)) return false;
    return true;
}

int check_batch(hj_batch b)
{
    if (!b || !reg_has(b) || b->magic != kBatchMagic)
        return set_err(HJ_ERR_HANDLE, "invalid or destroyed hj_batch handle");
    return HJ_OK;
}

// The form a batch runs a configuration in: XCD renumbering and reread
// apply to two-iteration passes only.
hj_config batch_form(hj_config c)
{
    if (c.tsteps == 0) c.tsteps = 1;
    if (c.tsteps != 2) {
        c.xcd_remap = 0;
        c.reread = 0;
    }
    return c;
}

}  // namespace

extern "C" {

int hj_batch_create(hj_batch* out, int dtype, int n, const int* nx, const int* ny, const int* nz,
                    void* stream)
{
    if (!out) return set_err(HJ_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (int rc = check_dtype(dtype)) return rc;
    if (n < 1 || !nx || !ny || !nz) return set_err(HJ_ERR_ARG, "need n >= 1 and shape arrays");
    return guarded([&]() -> int {
        hj_batch b = new hj_batch_s();
        b->dtype = dtype;
        b->n = n;
        b->L.resize(n);
        b->off.resize(n);
        b->uploaded.assign(n, 0u);
        size_t total = 0;
        for (int t = 0; t < n; ++t) {
            if (!make_layout(dtype, nx[t], ny[t], nz[t], b->L[t])) {
                delete b;
                return set_err(HJ_ERR_SHAPE, "instance %d: invalid shape %dx%dx%d", t, nx[t], ny[t], nz[t]);
            }
            b->off[t] = total;
            total += b->L[t].slab_bytes;
        }
        b->slab_bytes = total;
        b->cfg = batch_default(dtype);
        {
            hj_config c;
            if (cache_get("batch", dtype, batch_key(b->L), c) && config_supported(dtype, c) &&
                c.kernel != HJ_KERNEL_DIRECT && batch_fits(b, c)) {
                c.use_graph = 1;
                b->cfg = batch_form(c);
            }
        }
        try {
            dev_alloc(reinterpret_cast<void**>(&b->slab), total);
            if (stream) {
                b->stream = static_cast<hipStream_t>(stream);
            } else {
                stream_create(&b->stream);
                b->owns_stream = true;
            }
            stream_create(&b->cap);
            HIPCHK(hipEventCreate(&b->ev0));
            HIPCHK(hipEventCreate(&b->ev1));
            int dev = 0;
            HIPCHK(hipGetDevice(&dev));
            HIPCHK(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
            b->graphs.st = b->stream;
        } catch (...) {
            if (b->slab) dev_free(b->slab);
            if (b->owns_stream && b->stream) stream_destroy(b->stream);
            if (b->cap) stream_destroy(b->cap);
            if (b->ev0) (void)hipEventDestroy(b->ev0);
            if (b->ev1) (void)hipEventDestroy(b->ev1);
            delete b;
            throw;
        }
        reg_add(b);
        *out = b;
        return HJ_OK;
    });
}

}  // extern "C"

namespace {

int batch_upload(hj_batch b, int inst, int field, const void* src, bool src_f64)
{
    if (int rc = check_batch(b)) return rc;
    if (inst < 0 || inst >= b->n) return set_err(HJ_ERR_ARG, "instance %d out of range", inst);
    if (!src) return set_err(HJ_ERR_ARG, "host_src is NULL");
    if (host_mem(src) == HostMem::device) return set_err(HJ_ERR_ARG, "host_src is device memory, not a host array");
    if (field == HJ_WRK2) return set_err(HJ_ERR_ARG, "HJ_WRK2 cannot be uploaded");
    if (field < 0 || field >= HJ_WRK2) return set_err(HJ_ERR_ARG, "field %d out of range", field);
    return guarded([&]() -> int {
        if (field == HJ_P) {
            // the pair shares one parity: keep the instance's current buffer
            // and its partner identical so any parity is valid
            copy_in(b->L[inst], b->field(inst, HJ_P), src, src_f64, b->stream);
            copy_in(b->L[inst], b->field(inst, HJ_WRK2), src, src_f64, b->stream);
        } else {
            copy_in(b->L[inst], b->field(inst, field), src, src_f64, b->stream);
            gather_side(b->dtype, b->L[inst], field, b->origin(inst, field), b->side(inst), b->stream);
        }
        b->uploaded[inst] |= 1u << field;
        return HJ_OK;
    });
}

}  // namespace

extern "C" {

int hj_batch_upload(hj_batch b, int inst, int field, const void* src)
{
    return batch_upload(b, inst, field, src, false);
}

int hj_batch_upload_f64(hj_batch b, int inst, int field, const double* src)
{
    return batch_upload(b, inst, field, src, true);
}

int hj_batch_download(hj_batch b, int inst, int field, void* dst)
{
    if (int rc = check_batch(b)) return rc;
    if (inst < 0 || inst >= b->n) return set_err(HJ_ERR_ARG, "instance %d out of range", inst);
    if (!dst) return set_err(HJ_ERR_ARG, "host_dst is NULL");
    if (host_mem(dst) == HostMem::device) return set_err(HJ_ERR_ARG, "host_dst is device memory, not a host array");
    if (field < 0 || field >= HJ_NFIELDS) return set_err(HJ_ERR_ARG, "field %d out of range", field);
    return guarded([&]() -> int {
        int q = field;
        if (field == HJ_P || field == HJ_WRK2) q = b->parity ? HJ_WRK2 : HJ_P;
        copy_out(b->L[inst], b->field(inst, q), dst, b->stream);
        return HJ_OK;
    });
}

int hj_batch_sweep(hj_batch b, int n_iter, double omega, double* gosa_last, double* gosa_hist)
{
    if (int rc = check_batch(b)) return rc;
    if (n_iter < 0) return set_err(HJ_ERR_ARG, "n_iter %d < 0", n_iter);
    if (!b->all_uploaded()) return set_err(HJ_ERR_STATE, "not every input field of every instance is uploaded");
    if (n_iter == 0) return HJ_OK;
    return guarded([&]() -> int {
        b->reserve(n_iter);
        double* out = static_cast<double*>(b->gosa.p);
        HIPCHK(hipEventRecord(b->ev0, b->stream));
        b->run(n_iter, omega, out);
        HIPCHK(hipEventRecord(b->ev1, b->stream));
        const size_t nbytes = (size_t)n_iter * b->n * 8;
        b->host_gosa.ensure(nbytes);
        HIPCHK(hipMemcpyAsync(b->host_gosa.p, out, nbytes, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
        g_last_ms = ms;
        const double* hg = static_cast<const double*>(b->host_gosa.p);
        if (gosa_hist) memcpy(gosa_hist, hg, nbytes);
        if (gosa_last) memcpy(gosa_last, hg + (size_t)(n_iter - 1) * b->n, (size_t)b->n * 8);
        return HJ_OK;
    });
}

int hj_batch_residual(hj_batch b, double* gosa)
{
    if (int rc = check_batch(b)) return rc;
    if (!gosa) return set_err(HJ_ERR_ARG, "gosa is NULL");
    if (!b->all_uploaded()) return set_err(HJ_ERR_STATE, "not every input field of every instance is uploaded");
    return guarded([&]() -> int {
        b->reserve(1);
        double* pt = static_cast<double*>(b->part.p);
        double* out = static_cast<double*>(b->gosa.p);
        const BatchTiles& t = b->single_tiles();
        HIPCHK(b->launch_one(b->single_cfg(), t, b->parity, 0.0, false, pt, b->stream));
        HIPCHK(b->finalize(pt, t, 1, out, b->stream));
        b->host_gosa.ensure((size_t)b->n * 8);
        HIPCHK(hipMemcpyAsync(b->host_gosa.p, out, (size_t)b->n * 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        memcpy(gosa, b->host_gosa.p, (size_t)b->n * 8);
        return HJ_OK;
    });
}

int hj_batch_get_config(hj_batch b, hj_config* out)
{
    if (int rc = check_batch(b)) return rc;
    if (!out) return set_err(HJ_ERR_ARG, "out is NULL");
    *out = b->cfg;
    return HJ_OK;
}

int hj_batch_set_config(hj_batch b, const hj_config* cfg)
{
    if (int rc = check_batch(b)) return rc;
    if (int rc = validate_config(b->dtype, cfg)) return rc;
    if (cfg->kernel == HJ_KERNEL_DIRECT) return set_err(HJ_ERR_ARG, "batches run the march or flat kernel");
    if (!batch_fits(b, *cfg)) return set_err(HJ_ERR_ARG, "the flat kernel does not fit every instance");
    return guarded([&]() -> int {
        b->graphs.clear();
        b->cfg = batch_form(*cfg);
        return HJ_OK;
    });
}

}  // extern "C"

namespace {

// Tuning operations over a batch: the saved state is the whole slab (a
// second slab's worth of device memory, held for the session only). As for
// a single solve, an exception puts the slab and configuration back.
struct BatchTuning {
    hj_batch b;
    DevBuf save;
    Evaluator ev;
    hj_config keep;
    int par0;
    bool saved = false, finished = false;

    BatchTuning(const BatchTuning&) = delete;
    BatchTuning& operator=(const BatchTuning&) = delete;
    ~BatchTuning()
    {
        if (finished) return;
        try {
            if (saved) restore();
            (void)hipStreamSynchronize(b->stream);
            b->graphs.clear();
        } catch (...) {
        }
        (void)hipGetLastError();
        b->cfg = keep;
        b->tiled = false;
    }

    BatchTuning(hj_batch bb, int n_sweeps, int repeats) : b(bb)
    {
        keep = b->cfg;
        par0 = b->parity;
        save.ensure(b->slab_bytes);
        HIPCHK(hipMemcpyAsync(save.p, b->slab, b->slab_bytes, hipMemcpyDeviceToDevice, b->stream));
        saved = true;
        ev.n_sweeps = n_sweeps;
        ev.repeats = repeats;
        ev.kind = "batch";
        ev.dtype = b->dtype;
        ev.nx = b->n;
        ev.ops.st = b->stream;
        ev.ops.e0 = b->ev0;
        ev.ops.e1 = b->ev1;
        ev.ops.set = [this](const hj_config& c) {
            if (!batch_fits(b, c)) throw HipFail{hipErrorInvalidValue, "flat kernel does not fit", __LINE__};
            b->cfg = batch_form(c);
            b->cfg.use_graph = 1;
            b->reserve(ev.n_sweeps);
        };
        ev.ops.restore = [this] { restore(); };
        ev.ops.run = [this](int n) { b->run(n, 0.8, static_cast<double*>(b->gosa.p)); };
        ev.ops.result = [this] {
            // the current p of every instance (the partner buffer holds an
            // earlier iterate, which differs between one- and two-iteration passes)
            std::vector<std::pair<const void*, size_t>> r;
            for (int t = 0; t < b->n; ++t)
                r.emplace_back((const void*)b->field(t, b->parity ? HJ_WRK2 : HJ_P), b->L[t].field_bytes);
            return r;
        };
    }
    void restore()
    {
        HIPCHK(hipMemcpyAsync(b->slab, save.p, b->slab_bytes, hipMemcpyDeviceToDevice, b->stream));
        b->parity = par0;
    }
    int finish(const hj_config& win, double win_ms, hj_config* best, double* best_ms)
    {
        restore();
        HIPCHK(hipStreamSynchronize(b->stream));
        b->graphs.clear();
        finished = true;
        if (!std::isfinite(win_ms)) {
            b->cfg = keep;
            b->tiled = false;
            return set_err(HJ_ERR_TUNE, "no candidate configuration passed");
        }
        b->cfg = win;
        b->cfg.use_graph = keep.use_graph;
        cache_put("batch", b->dtype, batch_key(b->L), b->cfg, win_ms);
        if (best) *best = b->cfg;
        if (best_ms) *best_ms = win_ms;
        return HJ_OK;
    }
};

int batch_tunable(hj_batch b, int n_sweeps, int repeats)
{
    if (int rc = check_batch(b)) return rc;
    if (n_sweeps < 1 || repeats < 1) return set_err(HJ_ERR_ARG, "n_sweeps and repeats must be >= 1");
    if (!b->all_uploaded()) return set_err(HJ_ERR_STATE, "not every input field of every instance is uploaded");
    return HJ_OK;
}

std::vector<hj_config> batch_candidates(const hj_batch_s* b)
{
    const int dtype = b->dtype;
    std::vector<hj_config> out;
    for (int nw : {2, 4, 8})
        for (int ich : {2, 4, 8, 16, 32})
            for (int nt : {0, 1})
                for (int per : {0, 1}) {
                    hj_config c = batch_default(dtype);
                    c.kernel = HJ_KERNEL_FLAT;
                    c.bj = nw; c.vec = 1; c.ichunk = ich; c.nontemporal = nt; c.persistent = per;
                    if (config_supported(dtype, c) && batch_fits(b, c)) out.push_back(c);
                }
    const int vmax = dtype == HJ_F64 ? 2 : 4;
    for (int bj : {1, 2, 4, 8})
        for (int v = 1; v <= vmax; v *= 2)
            for (int ich : {2, 4, 8, 16, 32})
                for (int nt : {0, 1})
                    for (int per : {0, 1}) {
                        hj_config c = batch_default(dtype);
                        c.bj = bj; c.vec = v; c.ichunk = ich; c.nontemporal = nt; c.persistent = per;
                        if (config_supported(dtype, c)) out.push_back(c);
                    }
    // two iterations per pass, one workgroup per tile, with and without XCD
    // renumbering (without it measured 1% faster on batch64 FP32 at times)
    static const std::pair<int, int> kFusedShapes[] = {{1, 6}, {1, 8},  {1, 14}, {2, 6},  {2, 8},
                                                       {2, 12}, {4, 6}, {4, 14}, {4, 22}, {4, 30}};
    for (const auto& vb : kFusedShapes)
        for (int ich : {8, 12, 16, 24, 32, 48, 64, 128})
            for (int rr : {0, 1})
                for (int rm : {1, 0}) {
                    hj_config c = batch_default(dtype);
                    c.bj = vb.second; c.vec = vb.first; c.ichunk = ich; c.nontemporal = 0; c.tsteps = 2;
                    c.reread = rr; c.xcd_remap = rm;
                    if (config_supported(dtype, c)) out.push_back(c);
                }
    std::vector<hj_config> genes;
    add_gene_space(genes, dtype, 0, 0, 0, true);
    for (const hj_config& x : genes) {
        bool dup = false;
        for (const hj_config& y : out) dup = dup || same_config(x, y);
        if (!dup && (x.kernel != HJ_KERNEL_FLAT || batch_fits(b, x))) out.push_back(x);
    }
    return out;
}

}  // namespace

extern "C" {

int hj_batch_autotune(hj_batch b, int n_sweeps, int repeats, hj_config* best, double* best_ms)
{
    if (int rc = batch_tunable(b, n_sweeps, repeats)) return rc;
    return guarded([&]() -> int {
        BatchTuning tu(b, n_sweeps, repeats);
        hj_config refc = batch_default(b->dtype);
        refc.nontemporal = 0;
        tu.ev.eval(refc);
        hj_config win = tu.keep;
        double win_ms = INFINITY;
        for (const hj_config& c : batch_candidates(b)) {
            const double ms = tu.ev.eval(c);
            if (ms < win_ms) {
                win_ms = ms;
                win = c;
            }
        }
        return tu.finish(win, win_ms, best, best_ms);
    });
}

int hj_batch_autotune_ga(hj_batch b, int population, int generations, unsigned long long seed, double pc,
                         double pm, int n_sweeps, int repeats, hj_config* best, double* best_ms,
                         int* evaluations)
{
    if (int rc = batch_tunable(b, n_sweeps, repeats)) return rc;
    if (population < 1 || generations < 1 || !(pc >= 0.0 && pc <= 1.0) || !(pm >= 0.0 && pm <= 1.0))
        return set_err(HJ_ERR_ARG, "need population, generations >= 1 and 0 <= pc, pm <= 1");
    return guarded([&]() -> int {
        BatchTuning tu(b, n_sweeps, repeats);
        hj_config refc = batch_default(b->dtype);
        refc.nontemporal = 0;
        tu.ev.eval(refc);
        std::vector<std::pair<hj_config, double>> seen;
        auto time_of = [&](uint32_t g) -> double {
            hj_config c;
            if (!decode_gene(g, b->dtype, 0, 0, 0, true, c)) return hjga::kFailTime;
            for (auto& e : seen)
                if (same_config(e.first, c)) return e.second;
            const double ms = tu.ev.eval(c);
            const double t = std::isfinite(ms) ? ms * 1e-3 : hjga::kFailTime;
            seen.emplace_back(c, t);
            return t;
        };
        const hjga::Result r = hjga::run(kGeneBits, population, generations, seed, pc, pm, time_of);
        hj_config win = tu.keep;
        double win_ms = INFINITY;
        if (r.best_time < hjga::kFailTime && decode_gene(r.best_gene, b->dtype, 0, 0, 0, true, win))
            win_ms = r.best_time * 1e3;
        if (evaluations) *evaluations = r.evaluations;
        return tu.finish(win, win_ms, best, best_ms);
    });
}

int hj_ga_run(int gene_bits, int population, int generations, unsigned long long seed, double pc, double pm,
              const double* time_of_gene, unsigned* best_gene, double* best_time, unsigned* history,
              int* evaluations)
{
    if (gene_bits < 1 || gene_bits > 20 || population < 1 || generations < 1 || !time_of_gene ||
        !(pc >= 0.0 && pc <= 1.0) || !(pm >= 0.0 && pm <= 1.0))
        return set_err(HJ_ERR_ARG, "bad genetic search arguments");
    return guarded([&]() -> int {
        const hjga::Result r = hjga::run(gene_bits, population, generations, seed, pc, pm,
                                         [&](uint32_t g) { return time_of_gene[g]; });
        if (best_gene) *best_gene = r.best_gene;
        if (best_time) *best_time = r.best_time;
        if (evaluations) *evaluations = r.evaluations;
        if (history)
            for (size_t q = 0; q < r.history.size(); ++q) history[q] = r.history[q];
        return HJ_OK;
    });
}

int hj_gene_config(int dtype, int nx, int ny, int nz, int batch, unsigned gene, hj_config* out)
{
    if (!out) return set_err(HJ_ERR_ARG, "out is NULL");
    if (int rc = check_dtype(dtype)) return rc;
    hj_config c;
    if (!decode_gene(gene, dtype, nx, ny, nz, batch != 0, c))
        return set_err(HJ_ERR_ARG, "gene 0x%x names no configuration", gene);
    *out = c;
    return HJ_OK;
}

int hj_batch_destroy(hj_batch b)
{
    if (int rc = check_batch(b)) return rc;
    reg_del(b);
    (void)hipStreamSynchronize(b->stream);
    b->graphs.clear();
    b->part.release();
    b->gosa.release();
    b->host_gosa.release();
    b->tl.release();
    b->tl1.release();
    dev_free(b->slab);
    if (b->owns_stream) stream_destroy(b->stream);
    stream_destroy(b->cap);
    (void)hipEventDestroy(b->ev0);
    (void)hipEventDestroy(b->ev1);
    b->magic = 0;
    delete b;
    return HJ_OK;
}

}  // extern "C"
