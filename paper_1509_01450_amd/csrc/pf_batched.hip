// pf_batched.hip -- the many-disk forward map as one persistent launch, and
// the launch-shape autotuner.
//
// Batched path.  Every disk contributes work items (disk, pass, unit): pass A
// units (G rows of the phi transform), pass B units (G columns of the fused
// column pass), pass C units (G rows of the inverse phi transform).  The
// items of all disks are laid out in one list in dependency order -- every
// disk's A items, then every disk's B items, then every disk's C items -- and
// a persistent kernel's workgroups take them in that order from a global
// ticket counter.  A B item of disk d waits until all A items of d are done,
// a C item until all B items of d are done (per-disk counters, released with
// an agent-scope fence after the item's stores).  Because tickets are taken
// in dependency order, every item waited on was taken earlier by a workgroup
// that is already running and that itself only waits on earlier items, so
// the wait always ends; it is also bounded by a spin limit as a safeguard.
// The reset of the counters and the persistent kernel are captured once per
// batch signature in a HIP graph and replayed; the per-disk field pointers
// live in a device descriptor table that is refreshed when they change.
//
// Autotuner.  For each transform size and precision, candidate launch
// shapes (points per thread E -- the radix of the Stockham stages -- and
// transforms per workgroup G) are timed on the device with HIP events; the
// fastest is kept in memory and in a JSON file (PF_AUTOTUNE_CACHE, default
// ~/.cache/pf/autotune.json).  PF_AUTOTUNE=0 disables tuning.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "pass_bodies.hpp"
#include "pf_batched.hpp"

namespace pf {

// ===========================================================================
// Persistent batched kernel (FP32)
// ===========================================================================
constexpr int kBatchThreads = 256;
constexpr int kBatchE = 8;  // points per thread in every transform of a batch

struct DiskDesc {
    int n_r, n_phi, H, L, ldspec;
    int M;        // n_phi / 2
    int GA, GB;   // rows per A/C unit, columns per B unit
    int nA, nB;   // number of A and B units (dependency targets)
    float ca, c0, cn;
    const float *sigma;
    float *fr, *fp;
    cx<float> *S, *Zr, *Zp;
    const cx<float> *spec, *twN, *twL;
};

struct Item {
    int disk, pass, unit;
};

struct BatchCtl {
    int ticket;
    int timeouts;
};

// Wait until *ctr >= target.  The loop is uniform over the workgroup: every
// lane reads the counter with a relaxed agent-scope load (coherent across
// XCDs, no cache maintenance per poll) and the condition is taken from the
// first lane, so all waves leave together and see the same barriers.  Once
// the count is reached every wave performs one agent-scope acquire so the
// unit's loads see the producers' stores.  (Polling an acquire load would
// invalidate the XCD's L2 on every iteration.)
__device__ __forceinline__ void wait_count(int *ctr, int target, long spin_limit, BatchCtl *ctl) {
    long n = 0;
    bool timed_out = false;
    while (__builtin_amdgcn_readfirstlane(
               __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
        __builtin_amdgcn_s_sleep(8);
        if (++n > spin_limit) {
            timed_out = true;
            break;
        }
    }
    if (timed_out) atomicAdd(&ctl->timeouts, threadIdx.x == 0 ? 1 : 0);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// One size path per function (not inlined into the dispatch loop), so each
// transform size keeps the register allocation it needs alone.
template <int M>
__device__ __attribute__((noinline)) void run_rows(const Item &w, const DiskDesc &d, cx<float> *buf) {
    constexpr int TH = M / kBatchE;
    constexpr int G = kBatchThreads / TH;
    if (w.pass == 0)
        body_rows_r2c<float, M, kBatchE>(w.unit, G, buf, d.sigma, nullptr, d.n_r, d.n_r, d.S,
                                         nullptr, d.twN);
    else
        body_rows_c2r<float, M, kBatchE>(w.unit, G, buf, d.Zr, d.Zp, d.n_r, 2 * d.n_r, d.fr, d.fp,
                                         d.twN);
}

template <int L>
__device__ __attribute__((noinline)) void run_cols(const Item &w, const DiskDesc &d, cx<float> *buf) {
    constexpr int TH = L / kBatchE;
    constexpr int G = kBatchThreads / TH;
    body_cols_fwd<float, L, kBatchE>(w.unit, G, buf, d.S, d.Zr, d.Zp, d.spec, d.H, d.n_r,
                                     d.ldspec, d.ca, d.c0, d.cn, d.twL);
}

__global__ __launch_bounds__(kBatchThreads) void k_batched(const DiskDesc *__restrict__ disks,
                                                           const Item *__restrict__ items,
                                                           int n_items, BatchCtl *ctl,
                                                           int *doneA, int *doneB,
                                                           long spin_limit) {
    __shared__ cx<float> buf[padded_len(kBatchThreads * kBatchE)];
    __shared__ int s_it;
    for (;;) {
        // The dispatch loop is kept free of per-lane branches so that every
        // wave runs the same sequence of barriers: all lanes take part in
        // the atomics (only lane 0 of the workgroup adds a nonzero amount)
        // and the ticket is broadcast as a scalar (readfirstlane).
        const int tk = atomicAdd(&ctl->ticket, threadIdx.x == 0 ? 1 : 0);
        if (threadIdx.x == 0) s_it = tk;
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_it);
        __syncthreads();  // s_it read by all; LDS of the previous unit released
        if (it >= n_items) break;
        const Item w = items[it];
        const DiskDesc &d = disks[w.disk];
        if (w.pass == 1) wait_count(&doneA[w.disk], d.nA, spin_limit, ctl);
        if (w.pass == 2) wait_count(&doneB[w.disk], d.nB, spin_limit, ctl);
        if (w.pass == 1) {
            switch (d.L) {
                case 128: run_cols<128>(w, d, buf); break;
                case 256: run_cols<256>(w, d, buf); break;
                case 512: run_cols<512>(w, d, buf); break;
                case 1024: run_cols<1024>(w, d, buf); break;
                case 2048: run_cols<2048>(w, d, buf); break;
            }
        } else {
            switch (d.M) {
                case 64: run_rows<64>(w, d, buf); break;
                case 128: run_rows<128>(w, d, buf); break;
                case 256: run_rows<256>(w, d, buf); break;
                case 512: run_rows<512>(w, d, buf); break;
                case 1024: run_rows<1024>(w, d, buf); break;
                case 2048: run_rows<2048>(w, d, buf); break;
            }
        }
        if (w.pass < 2) {
            // every wave completes and releases its own stores at agent scope
            // (consumers may run on another XCD), then one lane publishes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            atomicAdd(w.pass == 0 ? &doneA[w.disk] : &doneB[w.disk], threadIdx.x == 0 ? 1 : 0);
        }
    }
}

__global__ void k_batch_reset(BatchCtl *ctl, int *done, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ctl->ticket = 0;
        ctl->timeouts = 0;
    }
    if (i < n) done[i] = 0;
}

namespace {

bool batch_size_ok(const Plan &p) {
    return p.opts.dtype == PF_F32 && p.M >= 64 && p.M <= 2048 && p.L >= 128 && p.L <= 2048;
}

struct BatchEntry {
    std::vector<int64_t> uids;
    int n = 0, n_items = 0, grid = 0;
    DiskDesc *d_desc = nullptr;
    Item *d_items = nullptr;
    BatchCtl *d_ctl = nullptr;
    int *d_done = nullptr;
    std::vector<DiskDesc> h_desc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = -1;

    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_desc) (void)hipFree(d_desc);
        if (d_items) (void)hipFree(d_items);
        if (d_ctl) (void)hipFree(d_ctl);
        if (d_done) (void)hipFree(d_done);
        exec = nullptr;
        graph = nullptr;
        d_desc = nullptr;
        d_items = nullptr;
        d_ctl = nullptr;
        d_done = nullptr;
    }
};

std::mutex g_batch_mu;
std::map<std::vector<int64_t>, BatchEntry> g_batches;

long spin_limit_env() {
    const char *s = getenv("PF_BATCH_SPIN_LIMIT");
    if (s && *s) return atol(s);
    return 1L << 21;  // about a second of polling: a safeguard, never reached
}

int make_entry(BatchEntry &e, const std::vector<const Plan *> &plans) {
    const int n = (int)plans.size();
    e.n = n;
    e.device = plans[0]->device;
    e.h_desc.resize(n);
    std::vector<Item> items;
    std::vector<Item> a, b, c;
    for (int k = 0; k < n; ++k) {
        const Plan &p = *plans[k];
        DiskDesc &d = e.h_desc[k];
        memset(&d, 0, sizeof(d));
        d.n_r = p.n_r;
        d.n_phi = p.n_phi;
        d.H = p.H;
        d.L = p.L;
        d.ldspec = p.ldspec;
        d.M = p.M;
        d.GA = kBatchThreads / (p.M / kBatchE);
        d.GB = kBatchThreads / (p.L / kBatchE);
        d.nA = (p.n_r + d.GA - 1) / d.GA;
        d.nB = (p.H + d.GB - 1) / d.GB;
        d.ca = (float)p.ca;
        d.c0 = (float)p.c0;
        d.cn = (float)p.cn;
        cx<float> *ws = (cx<float> *)p.ws;
        d.S = ws;
        d.Zr = ws + (size_t)p.n_r * p.H;
        d.Zp = d.Zr + (size_t)p.n_r * p.H;
        d.spec = (const cx<float> *)p.spec;
        d.twN = (const cx<float> *)p.twN;
        d.twL = (const cx<float> *)p.twL;
        const int nC = (2 * p.n_r + d.GA - 1) / d.GA;
        for (int u = 0; u < d.nA; ++u) a.push_back({k, 0, u});
        for (int u = 0; u < d.nB; ++u) b.push_back({k, 1, u});
        for (int u = 0; u < nC; ++u) c.push_back({k, 2, u});
    }
    items.insert(items.end(), a.begin(), a.end());
    items.insert(items.end(), b.begin(), b.end());
    items.insert(items.end(), c.begin(), c.end());
    e.n_items = (int)items.size();
    PF_HIP(hipMalloc(&e.d_desc, sizeof(DiskDesc) * n));
    PF_HIP(hipMalloc(&e.d_items, sizeof(Item) * items.size()));
    PF_HIP(hipMalloc(&e.d_ctl, sizeof(BatchCtl)));
    PF_HIP(hipMalloc(&e.d_done, sizeof(int) * 2 * n));
    PF_HIP(hipMemcpy(e.d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    // persistent grid: as many workgroups as stay resident
    int dev = 0, cus = 0, per_cu = 0;
    PF_HIP(hipGetDevice(&dev));
    PF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched, kBatchThreads, 0));
    if (per_cu < 1) per_cu = 1;
    e.grid = std::min(e.n_items, cus * per_cu);
    // capture reset + persistent kernel
    hipStream_t cs;
    PF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_batch_reset, dim3((2 * n + 255) / 256), dim3(256), 0, cs, e.d_ctl,
                           e.d_done, 2 * n);
        hipLaunchKernelGGL(k_batched, dim3(e.grid), dim3(kBatchThreads), 0, cs, e.d_desc,
                           e.d_items, e.n_items, e.d_ctl, e.d_done, e.d_done + n,
                           spin_limit_env());
        err = hipStreamEndCapture(cs, &e.graph);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (err != hipSuccess) {
        set_error("batch graph capture: %s", hipGetErrorString(err));
        return PF_EHIP;
    }
    return PF_OK;
}

}  // namespace

int batched_forces(const std::vector<const Plan *> &plans, const void *const *sigma,
                   void *const *f_r, void *const *f_phi, hipStream_t st) {
    const int n = (int)plans.size();
    std::vector<int64_t> key(n);
    for (int k = 0; k < n; ++k) {
        if (!batch_size_ok(*plans[k])) {
            set_error("batched path needs FP32 plans with 128 <= n_phi <= 4096 and "
                      "33 <= n_r <= 1024 (disk %d: %d x %d)",
                      k, plans[k]->n_r, plans[k]->n_phi);
            return PF_EUNSUPPORTED;
        }
        key[k] = plans[k]->uid;
    }
    {
        std::vector<int64_t> s = key;
        std::sort(s.begin(), s.end());
        if (std::adjacent_find(s.begin(), s.end()) != s.end()) {
            set_error("a plan appears twice in one batch (plans own their workspace)");
            return PF_EINVAL;
        }
    }
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto it = g_batches.find(key);
    if (it == g_batches.end()) {
        BatchEntry e;
        e.uids = key;
        int rc = make_entry(e, plans);
        if (rc) {
            e.release();
            return rc;
        }
        it = g_batches.emplace(key, e).first;
    }
    BatchEntry &e = it->second;
    bool changed = false;
    for (int k = 0; k < n; ++k) {
        DiskDesc &d = e.h_desc[k];
        if (d.sigma != sigma[k] || d.fr != f_r[k] || d.fp != f_phi[k]) {
            d.sigma = (const float *)sigma[k];
            d.fr = (float *)f_r[k];
            d.fp = (float *)f_phi[k];
            changed = true;
        }
    }
    if (changed) {
        // the descriptor table is read by the graph at replay time; the host
        // copy must outlive the transfer, so wait for it
        PF_HIP(hipMemcpyAsync(e.d_desc, e.h_desc.data(), sizeof(DiskDesc) * n,
                              hipMemcpyHostToDevice, st));
        PF_HIP(hipStreamSynchronize(st));
    }
    PF_HIP(hipGraphLaunch(e.exec, st));
    return PF_OK;
}

void batched_forget(int64_t uid) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    for (auto it = g_batches.begin(); it != g_batches.end();) {
        if (std::find(it->first.begin(), it->first.end(), uid) != it->first.end()) {
            it->second.release();
            it = g_batches.erase(it);
        } else {
            ++it;
        }
    }
}

// ===========================================================================
// Autotuner
// ===========================================================================
namespace {

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune;
bool g_tune_loaded = false;

std::string cache_path() {
    const char *p = getenv("PF_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char *h = getenv("HOME");
    if (!h || !*h) return "";
    return std::string(h) + "/.cache/pf/autotune.json";
}

// file format: one JSON object {"key": [E, G], ...}
void load_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    std::string s;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, n);
    fclose(f);
    size_t pos = 0;
    while (true) {
        size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        size_t b0 = s.find('[', q1);
        size_t b1 = s.find(']', b0 == std::string::npos ? q1 : b0);
        if (b0 == std::string::npos || b1 == std::string::npos) break;
        Shape sh;
        if (sscanf(s.c_str() + b0 + 1, "%d , %d", &sh.E, &sh.G) == 2) g_tune[key] = sh;
        pos = b1 + 1;
    }
}

void save_cache() {
    const std::string path = cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        // create the directory chain if needed (best effort)
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t k = 0;
    for (auto &kv : g_tune)
        fprintf(f, "  \"%s\": [%d, %d]%s\n", kv.first.c_str(), kv.second.E, kv.second.G,
                ++k < g_tune.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path.c_str());
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

template <class F>
float time_ms(F launch, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    for (int i = 0; i < 2; ++i)
        if (launch()) return -1.f;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.f;
    const int reps = 5;
    for (int i = 0; i < reps; ++i)
        if (launch()) return -1.f;
    if (hipEventRecord(e1, st) != hipSuccess) return -1.f;
    if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
    return ms / reps;
}

template <typename T>
void tune_t(Plan &p, hipStream_t st) {
    using C = cx<T>;
    const bool f64 = sizeof(T) == 8;
    const std::string pre = arch_name() + (f64 ? "|f64|" : "|f32|");
    const std::string krow = pre + "rows|M=" + std::to_string(p.M) + "|rows=" +
                             std::to_string(2 * p.n_r);
    const std::string kcol = pre + "cols|L=" + std::to_string(p.L) + "|H=" + std::to_string(p.H) +
                             "|n_r=" + std::to_string(p.n_r);
    const std::string kadj = pre + "adj|L=" + std::to_string(p.L) + "|H=" + std::to_string(p.H) +
                             "|n_r=" + std::to_string(p.n_r);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        load_cache();
        auto a = g_tune.find(krow), b = g_tune.find(kcol), c = g_tune.find(kadj);
        if (a != g_tune.end() && b != g_tune.end() && c != g_tune.end() &&
            valid_shape_rows(p.M, a->second, f64) && valid_shape_cols(p.L, b->second, f64) &&
            valid_shape_cols(p.L, c->second, f64)) {
            p.sched.rows = a->second;
            p.sched.cols = b->second;
            p.sched.cols_adj = c->second;
            return;
        }
    }
    T *x = nullptr;
    if (hipMalloc(&x, sizeof(T) * 3 * (size_t)p.n_r * p.n_phi) != hipSuccess) return;
    (void)hipMemsetAsync(x, 0, sizeof(T) * 3 * (size_t)p.n_r * p.n_phi, st);
    C *S = (C *)p.ws;
    C *Zr = S + (size_t)p.n_r * p.H, *Zp = Zr + (size_t)p.n_r * p.H;
    (void)hipMemsetAsync(p.ws, 0, sizeof(C) * 3 * (size_t)p.n_r * p.H, st);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // rows: forward R2C of n_r rows + inverse C2R of 2 n_r rows
    Shape best_r = p.sched.rows, best_c = p.sched.cols, best_a = p.sched.cols_adj;
    float tbest = 1e30f;
    for (int E : {4, 8, 16})
        for (int thr : {64, 128, 256, 512}) {
            if (E > p.M || (p.M / E) > thr) continue;
            Shape s{E, thr / (p.M / E)};
            if (!valid_shape_rows(p.M, s, f64)) continue;
            float t = time_ms(
                [&]() {
                    int rc = launch_rows_r2c<T>(p, x, nullptr, 1, p.n_r, S, nullptr,
                                                (const C *)p.twN, s, st);
                    if (!rc)
                        rc = launch_rows_c2r<T>(p, Zr, Zp, 2, p.n_r, x + (size_t)p.n_r * p.n_phi,
                                                x + 2 * (size_t)p.n_r * p.n_phi,
                                                (const C *)p.twN, s, st);
                    return rc;
                },
                st, e0, e1);
            if (t > 0 && t < tbest) {
                tbest = t;
                best_r = s;
            }
        }
    tbest = 1e30f;
    for (int E : {8, 16})
        for (int thr : {64, 128, 256, 512}) {
            if (E > p.L || (p.L / E) > thr) continue;
            Shape s{E, thr / (p.L / E)};
            if (!valid_shape_cols(p.L, s, f64)) continue;
            float t = time_ms(
                [&]() {
                    return launch_cols_fwd<T>(p, S, Zr, Zp, (const C *)p.spec, (const C *)p.twL,
                                              s, st);
                },
                st, e0, e1);
            if (t > 0 && t < tbest) {
                tbest = t;
                best_c = s;
            }
        }
    tbest = 1e30f;
    for (int E : {8, 16})
        for (int thr : {64, 128, 256, 512}) {
            if (E > p.L || (p.L / E) > thr) continue;
            Shape s{E, thr / (p.L / E)};
            if (!valid_shape_cols(p.L, s, f64)) continue;
            float t = time_ms(
                [&]() {
                    return launch_cols_adj<T>(p, S, Zr, Zp, (const C *)p.spec, (const C *)p.twL,
                                              s, st);
                },
                st, e0, e1);
            if (t > 0 && t < tbest) {
                tbest = t;
                best_a = s;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(x);
    clear_error();
    p.sched.rows = best_r;
    p.sched.cols = best_c;
    p.sched.cols_adj = best_a;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[krow] = best_r;
    g_tune[kcol] = best_c;
    g_tune[kadj] = best_a;
    save_cache();
}

}  // namespace

void autotune_plan(Plan &p, hipStream_t st) {
    const char *e = getenv("PF_AUTOTUNE");
    if (e && e[0] == '0') return;
    if (p.opts.dtype == PF_F64)
        tune_t<double>(p, st);
    else
        tune_t<float>(p, st);
}

}  // namespace pf
