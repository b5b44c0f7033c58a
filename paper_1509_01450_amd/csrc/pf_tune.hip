// pf_tune.hip -- the launch-shape autotuner.  For each transform size and
// precision, candidate launch shapes (points per thread E -- the radix of
// the Stockham stages -- and transforms per workgroup G) are timed on the
// device with HIP events; the fastest is kept in memory and in a JSON file
// (PF_AUTOTUNE_CACHE, default ~/.cache/pf/autotune.json).  PF_AUTOTUNE=0
// disables tuning.
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "pf_batched.hpp"

namespace pf {

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

// Mean duration (ms) of one launch: the best of three runs of 20
// back-to-back launches after three warm-up launches (candidates a few
// percent apart are told apart reliably).  A failed launch or event call
// returns its status; *ms is then untouched.
template <class F>
int time_ms(F launch, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float *ms) {
    for (int i = 0; i < 3; ++i) {
        const int rc = launch();
        if (rc) return rc;
    }
    const int reps = 20;
    float best = -1.f;
    for (int trial = 0; trial < 3; ++trial) {
        PF_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < reps; ++i) {
            const int rc = launch();
            if (rc) return rc;
        }
        PF_HIP(hipEventRecord(e1, st));
        PF_HIP(hipEventSynchronize(e1));
        float t = 0;
        PF_HIP(hipEventElapsedTime(&t, e0, e1));
        if (best < 0.f || t < best) best = t;
    }
    *ms = best / reps;
    return PF_OK;
}

// Device resources of one tuning run, released on every return path.
struct TuneScratch {
    void *x = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        if (x) (void)hipFree(x);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <typename T>
int tune_t(Plan &p, hipStream_t st) {
    using C = cx<T>;
    const bool f64 = sizeof(T) == 8;
    const std::string pre = arch_name() + (f64 ? "|f64|" : "|f32|");
    const std::string krow = pre + "rows1|M=" + std::to_string(p.M) + "|rows=" +
                             std::to_string(p.n_r);
    const std::string krow2 = pre + "rows2|M=" + std::to_string(p.M) + "|rows=" +
                              std::to_string(p.n_r);
    // the column kernels of slope order 4 are other kernels: their own keys
    const std::string so = p.so == 4 ? "|so=4" : "";
    const std::string kcol = pre + "cols|L=" + std::to_string(p.L) + "|H=" + std::to_string(p.H) +
                             "|n_r=" + std::to_string(p.n_r) + so;
    const std::string kadj = pre + "adj|L=" + std::to_string(p.L) + "|H=" + std::to_string(p.H) +
                             "|n_r=" + std::to_string(p.n_r) + so;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        load_cache();
        auto a = g_tune.find(krow), a2 = g_tune.find(krow2), b = g_tune.find(kcol),
             c = g_tune.find(kadj);
        if (a != g_tune.end() && a2 != g_tune.end() && b != g_tune.end() && c != g_tune.end() &&
            valid_shape_rows(p.M, a->second, f64) && valid_shape_rows(p.M, a2->second, f64) &&
            valid_shape_cols(p.L, b->second, f64) && valid_shape_cols(p.L, c->second, f64)) {
            p.sched.rows = a->second;
            p.sched.rows2 = a2->second;
            p.sched.cols = b->second;
            p.sched.cols_adj = c->second;
            return PF_OK;
        }
    }
    TuneScratch ts;
    const size_t xbytes = sizeof(T) * 3 * (size_t)p.n_r * p.n_phi;
    PF_HIP(hipMalloc(&ts.x, xbytes));
    T *x = (T *)ts.x;
    PF_HIP(hipMemsetAsync(x, 0, xbytes, st));
    C *S = (C *)p.ws;                        // forward: S, then (Zr, Zp) pairs
    C *Z = S + (size_t)p.n_r * p.H;
    C *D = S + 2 * (size_t)p.n_r * p.H;      // transpose: (Vr, Vp) pairs at S, then D
    PF_HIP(hipMemsetAsync(p.ws, 0, sizeof(C) * 3 * (size_t)p.n_r * p.H, st));
    PF_HIP(hipEventCreate(&ts.e0));
    PF_HIP(hipEventCreate(&ts.e1));
    // rows: the one-channel forward R2C and the two-channel inverse C2R of
    // n_r rows, each on its own (they stand for the one- and two-channel row
    // transforms of both directions)
    Shape best_r = p.sched.rows, best_r2 = p.sched.rows2, best_c = p.sched.cols,
          best_a = p.sched.cols_adj;
    // Bring the GPU to its working clocks first (a few ms of the default
    // shapes): timed right after the plan build, the first candidates ran at
    // lower clocks and lost to later ones they beat in steady state.  Each
    // candidate set is then swept twice, keeping every candidate's best time.
    for (int i = 0; i < 100; ++i) {
        int rc = launch_rows_c2r<T>(p, Z, p.n_r, x + (size_t)p.n_r * p.n_phi,
                                    x + 2 * (size_t)p.n_r * p.n_phi, (const C *)p.twN,
                                    p.sched.rows2, st, p.gscale);
        if (!rc)
            rc = launch_cols_fwd<T>(p, S, Z, (const C *)p.spec, (const C *)p.twL, p.sched.cols,
                                    st, p.gscale);
        if (rc) return rc;
    }
    PF_HIP(hipStreamSynchronize(st));
    float tbest = 1e30f, tbest2 = 1e30f, t = 0.f;
    int rc = PF_OK;
    for (int sweep = 0; sweep < 2; ++sweep)
        for (int E : {2, 4, 8, 16})
            for (int thr : {64, 128, 256, 512}) {
                if (E > row_sub(p.M) || row_threads(p.M, E) > thr) continue;
                Shape s{E, thr / row_threads(p.M, E)};
                if (!valid_shape_rows(p.M, s, f64)) continue;
                rc = time_ms(
                    [&]() {
                        return launch_rows_r2c<T>(p, x, nullptr, p.n_r, S, (const C *)p.twN, s,
                                                  st, p.gscale);
                    },
                    st, ts.e0, ts.e1, &t);
                if (rc) return rc;
                if (t < tbest) {
                    tbest = t;
                    best_r = s;
                }
                rc = time_ms(
                    [&]() {
                        return launch_rows_c2r<T>(p, Z, p.n_r, x + (size_t)p.n_r * p.n_phi,
                                                  x + 2 * (size_t)p.n_r * p.n_phi,
                                                  (const C *)p.twN, s, st, p.gscale);
                    },
                    st, ts.e0, ts.e1, &t);
                if (rc) return rc;
                if (t < tbest2) {
                    tbest2 = t;
                    best_r2 = s;
                }
            }
    for (int adj = 0; adj < 2; ++adj) {
        tbest = 1e30f;
        Shape &best = adj ? best_a : best_c;
        for (int sweep = 0; sweep < 2; ++sweep)
            for (int E : {8, 16})
                for (int thr : {64, 128, 256, 512}) {
                    if (E > p.L || (p.L / E) > thr) continue;
                    Shape s{E, thr / (p.L / E)};
                    if (!valid_shape_cols(p.L, s, f64)) continue;
                    rc = time_ms(
                        [&]() {
                            return adj ? launch_cols_adj<T>(p, S, D, (const C *)p.spec,
                                                            (const C *)p.twL, s, st, p.gscale)
                                       : launch_cols_fwd<T>(p, S, Z, (const C *)p.spec,
                                                            (const C *)p.twL, s, st, p.gscale);
                        },
                        st, ts.e0, ts.e1, &t);
                    if (rc) return rc;
                    if (t < tbest) {
                        tbest = t;
                        best = s;
                    }
                }
    }
    // the timing runs left notes in the scale words: clear them for the
    // first call
    if (p.gscale) PF_HIP(hipMemsetAsync(p.gscale, 0, 2 * kScaleSet * sizeof(unsigned), st));
    PF_HIP(hipStreamSynchronize(st));
    p.sched.rows = best_r;
    p.sched.rows2 = best_r2;
    p.sched.cols = best_c;
    p.sched.cols_adj = best_a;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[krow] = best_r;
    g_tune[krow2] = best_r2;
    g_tune[kcol] = best_c;
    g_tune[kadj] = best_a;
    save_cache();
    return PF_OK;
}

}  // namespace

int autotune_plan(Plan &p, hipStream_t st) {
    const char *e = getenv("PF_AUTOTUNE");
    if (e && e[0] == '0') return PF_OK;
    return p.opts.dtype == PF_F64 ? tune_t<double>(p, st) : tune_t<float>(p, st);
}

}  // namespace pf
