// pf_api.hip -- host side of the C ABI declared in include/pf.h: argument
// validation, plan geometry (Sec. 3.2.1), build orchestration and the launch
// sequences of the forward map and its transpose.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "pf_batched.hpp"
#include "pf_common.hpp"

namespace pf {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }

void twiddles_host(int n, std::vector<double> &re, std::vector<double> &im) {
    re.resize(n);
    im.resize(n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int j = 0; j < n; ++j) {
        // reduce to the first octant by symmetry so every entry is accurate
        const long double a = two_pi * (long double)j / (long double)n;
        re[j] = (double)cosl(a);
        im[j] = (double)(-sinl(a));
    }
    // exact values at the quarter points
    for (int q = 0; q < 4; ++q) {
        if ((long)q * n % 4) continue;
        const int j = (int)((long)q * n / 4);
        static const double c[4] = {1, 0, -1, 0}, s[4] = {0, -1, 0, 1};
        re[j] = c[q];
        im[j] = s[q];
    }
}

int upload_twiddles(int n, bool f64, void **dst) {
    std::vector<double> re, im;
    twiddles_host(n, re, im);
    const size_t bytes = (size_t)n * (f64 ? 16 : 8);
    std::vector<unsigned char> buf(bytes);
    for (int j = 0; j < n; ++j) {
        if (f64) {
            double v[2] = {re[j], im[j]};
            memcpy(&buf[(size_t)j * 16], v, 16);
        } else {
            float v[2] = {(float)re[j], (float)im[j]};
            memcpy(&buf[(size_t)j * 8], v, 8);
        }
    }
    PF_HIP(hipMalloc(dst, bytes));
    PF_HIP(hipMemcpy(*dst, buf.data(), bytes, hipMemcpyHostToDevice));
    return PF_OK;
}

Schedule default_schedule(int n_phi, int L, bool f64) {
    Schedule s;
    const int M = n_phi / 2;
    if (!is_pow2_int(M)) {   // M = Q P: 4 points per thread (2 for Q = 9)
        s.rows.E = row_factor(M) == 9 ? 2 : 4;
    } else {
        s.rows.E = M >= 2048 ? 16 : (M < 8 ? M : 8);
        if (s.rows.E < 4) s.rows.E = 4;
    }
    {
        const int th = row_threads(M, s.rows.E);
        s.rows.G = th >= 256 ? 1 : 256 / th;
        while (s.rows.G > 1 && !valid_shape_rows(M, s.rows, f64)) s.rows.G /= 2;
    }
    s.rows2 = s.rows;
    // column pass: 16 points per thread in FP32 from L = 2048 on (fewer LDS
    // exchanges, two columns per workgroup), 8 otherwise; the transpose pass
    // holds two input channels and takes 8
    s.cols.E = (!f64 && L >= 2048) || L >= 4096 ? 16 : 8;
    s.cols_adj.E = L >= 4096 ? 16 : 8;
    for (Shape *c : {&s.cols, &s.cols_adj}) {
        const int th = L / c->E;
        c->G = th >= 256 ? 1 : 256 / th;
        while (c->G > 1 && !valid_shape_cols(L, *c, f64)) c->G /= 2;
    }
    return s;
}

static int64_t next_uid() {
    static std::mutex mu;
    static int64_t uid = 0;
    std::lock_guard<std::mutex> g(mu);
    return ++uid;
}

static void free_plan_device(Plan *p) {
    if (p->spec) (void)hipFree(p->spec);
    if (p->twN) (void)hipFree(p->twN);
    if (p->twL) (void)hipFree(p->twL);
    if (p->ws) (void)hipFree(p->ws);
    if (p->tables) (void)hipFree(p->tables);
    if (p->wspec) (void)hipFree(p->wspec);
    if (p->wws) (void)hipFree(p->wws);
    p->spec = p->twN = p->twL = p->ws = p->wspec = p->wws = nullptr;
    p->gscale = nullptr;
    p->tables = nullptr;
    p->built = false;
}

static int device_present() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        set_error("no GPU device available");
        return PF_ENODEV;
    }
    return PF_OK;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace pf

using pf::Plan;

struct pf_plan_s {
    Plan p;
};

namespace {

int check_call(pf_plan h, const void *a, const void *b, const void *c) {
    if (!h) {
        pf::set_error("null plan");
        return PF_EINVAL;
    }
    if (!a || !b || !c) {
        pf::set_error("null field pointer");
        return PF_EINVAL;
    }
    if (!h->p.built) {
        pf::set_error("plan not built (call pf_kernels_build first)");
        return PF_ESTATE;
    }
    return PF_OK;
}

// Forward map: pass A on the n_in source rows, pass B, the origin wedges'
// terms (plans with wedges), pass C on the n_r destination rows.
template <typename T>
int forces_t(const Plan &p, const T *sigma, const T *sigma_w, T *fr, T *fp, hipStream_t st) {
    using C = pf::cx<T>;
    C *S = (C *)p.ws;
    C *Z = S + (size_t)p.n_in * p.H;   // (Zr, Zp) pairs
    unsigned *g = p.gscale;   // the forward map's scale words
    // plans with wedges: the wedge row's transform rides in pass A's launch
    C *wrow = p.wedges ? (C *)p.wws : nullptr;
    int rc = pf::launch_rows_r2c<T>(p, sigma, nullptr, p.n_in, S, (const C *)p.twN, p.sched.rows,
                                    st, g, p.wedges ? sigma_w : nullptr, wrow);
    if (rc) return rc;
    rc = pf::launch_cols_fwd<T>(p, S, Z, (const C *)p.spec, (const C *)p.twL, p.sched.cols, st,
                                g);
    if (rc) return rc;
    if (p.wedges) {
        rc = pf::launch_wedge_terms<T>(p, S, wrow, Z, st, g);
        if (rc) return rc;
    }
    return pf::launch_rows_c2r<T>(p, Z, p.n_r, fr, fp, (const C *)p.twN, p.sched.rows2, st, g,
                                  p.col0);
}

// Transpose: pass A on the n_r destination rows of both cotangents, the
// transposed column pass to the n_in source rows, pass C on those; plans
// with wedges add the wedges' sums from the same row spectra before pass C,
// whose launch also transforms the wedge row.
template <typename T>
int backward_t(const Plan &p, const T *gr, const T *gp, T *gs, T *gw, hipStream_t st) {
    using C = pf::cx<T>;
    C *V = (C *)p.ws;                        // (Vr, Vp) pairs, n_r rows
    C *D = V + 2 * (size_t)p.n_r * p.H;      // n_in rows
    unsigned *g = p.gscale ? p.gscale + pf::kScaleSet : nullptr;   // the transpose's words
    int rc = pf::launch_rows_r2c<T>(p, gr, gp, p.n_r, V, (const C *)p.twN, p.sched.rows2, st, g);
    if (rc) return rc;
    rc = pf::launch_cols_adj<T>(p, V, D, (const C *)p.spec, (const C *)p.twL, p.sched.cols_adj,
                                st, g);
    if (rc) return rc;
    if (p.wedges) {
        rc = pf::launch_wedge_adjoint_sums<T>(p, V, D, st, g);
        if (rc) return rc;
    }
    return pf::launch_rows_c2r<T>(p, D, p.n_in, gs, nullptr, (const C *)p.twN, p.sched.rows, st,
                                  g, -p.col0, p.wedges ? (const C *)p.wws : nullptr,
                                  p.wedges ? gw : nullptr);
}

template <typename T>
int timed_t(const Plan &p, bool bwd, const void *in0, const void *in1, void *out0, void *out1,
            int reps, hipStream_t st, hipEvent_t *ev) {
    using C = pf::cx<T>;
    C *W0 = (C *)p.ws;
    C *W1 = W0 + (size_t)p.n_in * p.H;      // forward: S = W0, Z = W1
    C *W2 = W0 + 2 * (size_t)p.n_r * p.H;   // transpose: V = W0, D = W2
    int rc = PF_OK;
    unsigned *g = p.gscale ? p.gscale + (bwd ? pf::kScaleSet : 0) : nullptr;
    PF_HIP(hipEventRecord(ev[0], st));
    for (int k = 0; k < reps && !rc; ++k)
        rc = pf::launch_rows_r2c<T>(p, (const T *)in0, bwd ? (const T *)in1 : nullptr,
                                    bwd ? p.n_r : p.n_in, W0, (const C *)p.twN,
                                    bwd ? p.sched.rows2 : p.sched.rows, st, g);
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[1], st));
    for (int k = 0; k < reps && !rc; ++k) {
        if (!bwd)
            rc = pf::launch_cols_fwd<T>(p, W0, W1, (const C *)p.spec, (const C *)p.twL,
                                        p.sched.cols, st, g);
        else
            rc = pf::launch_cols_adj<T>(p, W0, W2, (const C *)p.spec, (const C *)p.twL,
                                        p.sched.cols_adj, st, g);
    }
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[2], st));
    for (int k = 0; k < reps && !rc; ++k) {
        if (!bwd)
            rc = pf::launch_rows_c2r<T>(p, W1, p.n_r, (T *)out0, (T *)out1, (const C *)p.twN,
                                        p.sched.rows2, st, g, p.col0);
        else
            rc = pf::launch_rows_c2r<T>(p, W2, p.n_in, (T *)out0, nullptr, (const C *)p.twN,
                                        p.sched.rows, st, g, -p.col0);
    }
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[3], st));
    return PF_OK;
}

}  // namespace

extern "C" {

const char *pf_last_error(void) { return pf::g_err; }

const char *pf_version(void) { return "pf 0.1 (gfx950)"; }

void pf_build_opts_default(pf_build_opts *o) {
    if (!o) return;
    o->dtype = PF_F32;
    o->n_tpz = 19;
    o->cover_per = 10;
    o->table_mode = PF_TABLE_SIM;
    o->self_mode = PF_SELF_CARTESIAN;
    o->method = PF_METHOD_SIM;
    o->keep_tables = 0;
    o->slope_order = 2;
}

pf_plan pf_plan_create(int n_r, int n_phi, double r_min, double r_max) {
    pf::clear_error();
    if (n_r < 4 || n_r > 4096) {
        pf::set_error("n_r = %d outside [4, 4096]", n_r);
        return nullptr;
    }
    const bool three = n_phi % 6 == 0 && pf::is_pow2(n_phi / 6);
    const bool nine = n_phi % 18 == 0 && pf::is_pow2(n_phi / 18);
    if (!((pf::is_pow2(n_phi) && n_phi >= 8 && n_phi <= 8192) ||
          (three && n_phi >= 24 && n_phi <= 6144) || (nine && n_phi >= 72 && n_phi <= 4608))) {
        pf::set_error("n_phi = %d must be a power of two in [8, 8192], three times one in "
                      "[24, 6144] or nine times one in [72, 4608]", n_phi);
        return nullptr;
    }
    if (!std::isfinite(r_min) || !std::isfinite(r_max) || !(r_min > 0) || !(r_max > r_min)) {
        pf::set_error("need finite 0 < r_min < r_max (got %g, %g)", r_min, r_max);
        return nullptr;
    }
    pf_plan_s *h = new (std::nothrow) pf_plan_s();
    if (!h) {
        pf::set_error("out of host memory");
        return nullptr;
    }
    Plan &p = h->p;
    p.n_r = n_r;
    p.n_in = n_r;
    p.s0 = 0;
    p.n_phi = n_phi;
    p.M = n_phi / 2;
    p.H = n_phi / 2;   // packed half spectrum: bins 0 and n_phi/2 share column 0
    int L = 8;
    while (L < 2 * n_r) L *= 2;  // zero padding: any L >= 2 n_r - 1 is exact
    p.L = L;
    p.ldspec = L / 2 + 1;
    p.r_min = r_min;
    p.r_max = r_max;
    p.beta = std::pow(r_max / r_min, 1.0 / n_r);
    p.dphi = 2.0 * M_PI / n_phi;
    // g = r_i delta^r_i:  r_i / (r_{i+1} - r_{i-1}) = 1 / (beta - 1/beta), and
    // the one-sided ends 1 / (beta - 1), 1 / (1 - 1/beta)
    p.ca = 1.0 / (p.beta - 1.0 / p.beta);
    p.c0 = 1.0 / (p.beta - 1.0);
    p.cn = 1.0 / (1.0 - 1.0 / p.beta);
    pf_build_opts_default(&p.opts);
    p.uid = pf::next_uid();
    return h;
}

pf_plan pf_plan_create_patches(int n_src, int src_row0, int n_dst, int n_phi, double r_min,
                               double r_max, int wedges) {
    pf::clear_error();
    if (n_src < 4 || n_src > 4096) {
        pf::set_error("n_src = %d outside [4, 4096]", n_src);
        return nullptr;
    }
    if (src_row0 < -65536 || src_row0 > 65536) {
        pf::set_error("src_row0 = %d outside [-65536, 65536]", src_row0);
        return nullptr;
    }
    if (wedges && src_row0 > 0) {
        pf::set_error("origin wedges need the source patch to start at or below r_min "
                      "(src_row0 <= 0, got %d)", src_row0);
        return nullptr;
    }
    pf_plan h = pf_plan_create(n_dst, n_phi, r_min, r_max);
    if (!h) return nullptr;
    Plan &p = h->p;
    p.n_in = n_src;
    p.s0 = src_row0;
    p.patch = true;
    p.wedges = wedges != 0;
    int L = 8;
    while (L < 2 * n_src || L < 2 * n_dst) L *= 2;
    p.L = L;
    p.ldspec = L / 2 + 1;
    return h;
}

int pf_plan_set_src_col0(pf_plan h, int src_col0) {
    pf::clear_error();
    if (!h) {
        pf::set_error("null plan");
        return PF_EINVAL;
    }
    if (!h->p.patch) {
        pf::set_error("an azimuthal turn needs a patch plan");
        return PF_EINVAL;
    }
    const int n = h->p.n_phi;
    h->p.col0 = ((src_col0 % n) + n) % n;
    return PF_OK;
}

void pf_plan_destroy(pf_plan h) {
    if (!h) return;
    pf::batched_forget(h->p.uid);
    pf::free_plan_device(&h->p);
    delete h;
}

int pf_plan_geometry(pf_plan h, double *r_centres, double *r_edges, double *dphi) {
    pf::clear_error();
    if (!h) {
        pf::set_error("null plan");
        return PF_EINVAL;
    }
    const Plan &p = h->p;
    for (int i = 0; i <= p.n_r; ++i) {
        const double lo = p.r_min * std::pow(p.beta, i);
        if (r_edges) r_edges[i] = lo;
        if (r_centres && i < p.n_r) {
            const double hi = p.r_min * std::pow(p.beta, i + 1);
            r_centres[i] = 0.5 * (lo + hi);
        }
    }
    if (dphi) *dphi = p.dphi;
    return PF_OK;
}

int pf_plan_selfcell(pf_plan h, double out[3]) {
    pf::clear_error();
    if (!h || !out) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    if (!h->p.built) {
        pf::set_error("plan not built");
        return PF_ESTATE;
    }
    for (int q = 0; q < 3; ++q) out[q] = h->p.selfk[q];
    return PF_OK;
}

int pf_plan_schedule(pf_plan h, int out[8]) {
    pf::clear_error();
    if (!h || !out) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    if (!h->p.built) {
        pf::set_error("plan not built");
        return PF_ESTATE;
    }
    const pf::Schedule &s = h->p.sched;
    out[0] = s.rows.E;
    out[1] = s.rows.G;
    out[2] = s.rows2.E;
    out[3] = s.rows2.G;
    out[4] = s.cols.E;
    out[5] = s.cols.G;
    out[6] = s.cols_adj.E;
    out[7] = s.cols_adj.G;
    return PF_OK;
}

int pf_plan_set_schedule(pf_plan h, const int in[8]) {
    pf::clear_error();
    if (!h || !in) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    pf::Plan &p = h->p;
    // the shapes are checked first (against the plan's current precision),
    // so a bad shape is refused whether or not the plan is built
    const bool f64 = p.opts.dtype == PF_F64;
    const pf::Shape r1{in[0], in[1]}, r2{in[2], in[3]}, c{in[4], in[5]}, a{in[6], in[7]};
    if (!pf::valid_shape_rows(p.M, r1, f64) || !pf::valid_shape_rows(p.M, r2, f64)) {
        pf::set_error("row shapes (%d, %d), (%d, %d) do not fit %d-point row transforms", r1.E,
                      r1.G, r2.E, r2.G, p.M);
        return PF_EINVAL;
    }
    if (!pf::valid_shape_cols(p.L, c, f64) || !pf::valid_shape_cols(p.L, a, f64)) {
        pf::set_error("column shapes (%d, %d), (%d, %d) do not fit %d-point column transforms",
                      c.E, c.G, a.E, a.G, p.L);
        return PF_EINVAL;
    }
    if (!p.built) {
        pf::set_error("plan not built");
        return PF_ESTATE;
    }
    pf::batched_forget(p.uid);   // batches group disks by their launch shapes
    p.sched.rows = r1;
    p.sched.rows2 = r2;
    p.sched.cols = c;
    p.sched.cols_adj = a;
    return PF_OK;
}

int pf_plan_tables(pf_plan h, double *dst) {
    pf::clear_error();
    if (!h || !dst) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    const Plan &p = h->p;
    if (!p.built || !p.tables) {
        pf::set_error("plan not built with keep_tables");
        return PF_ESTATE;
    }
    const int rows = p.n_in + p.n_r - 1;
    for (int k = 0; k < 6; ++k)
        for (int ir = 0; ir < rows; ++ir) {
            const int m = ir - (p.n_in - 1);
            const int row = (m % p.L + p.L) % p.L;
            PF_HIP(hipMemcpy(dst + ((size_t)k * rows + ir) * p.n_phi,
                             p.tables + ((size_t)k * p.L + row) * p.n_phi,
                             (size_t)p.n_phi * sizeof(double), hipMemcpyDeviceToHost));
        }
    return PF_OK;
}

int pf_kernels_build(pf_plan h, const pf_build_opts *opts, void *stream) {
    pf::clear_error();
    if (!h) {
        pf::set_error("null plan");
        return PF_EINVAL;
    }
    pf_build_opts o;
    if (opts)
        o = *opts;
    else
        pf_build_opts_default(&o);
    if (o.dtype != PF_F32 && o.dtype != PF_F64) {
        pf::set_error("dtype must be PF_F32 or PF_F64");
        return PF_EINVAL;
    }
    if (o.table_mode != PF_TABLE_SIM && o.table_mode != PF_TABLE_EXACT) {
        pf::set_error("table_mode must be PF_TABLE_SIM or PF_TABLE_EXACT");
        return PF_EINVAL;
    }
    if (o.self_mode != PF_SELF_CARTESIAN && o.self_mode != PF_SELF_EXACT) {
        pf::set_error("self_mode must be PF_SELF_CARTESIAN or PF_SELF_EXACT");
        return PF_EINVAL;
    }
    if (o.method != PF_METHOD_SIM && o.method != PF_METHOD_PARTICLE &&
        o.method != PF_METHOD_PARTICLE_PLUS) {
        pf::set_error("method must be PF_METHOD_SIM, PF_METHOD_PARTICLE or "
                      "PF_METHOD_PARTICLE_PLUS");
        return PF_EINVAL;
    }
    if (o.method == PF_METHOD_SIM && o.table_mode == PF_TABLE_SIM &&
        (o.n_tpz < 1 || o.n_tpz > 1024)) {
        pf::set_error("n_tpz = %d outside [1, 1024]", o.n_tpz);
        return PF_EINVAL;
    }
    if (o.method != PF_METHOD_PARTICLE && o.self_mode == PF_SELF_CARTESIAN &&
        (o.cover_per < 1 || o.cover_per > 64)) {
        pf::set_error("cover_per = %d outside [1, 64]", o.cover_per);
        return PF_EINVAL;
    }
    if (o.slope_order != 2 && o.slope_order != 4) {
        pf::set_error("slope_order must be 2 or 4 (got %d)", o.slope_order);
        return PF_EINVAL;
    }
    if (o.slope_order == 4 && h->p.patch) {
        pf::set_error("slope order 4 is not built for patch plans");
        return PF_EUNSUPPORTED;
    }
    int rc = pf::device_present();
    if (rc) return rc;
    Plan &p = h->p;
    pf::batched_forget(p.uid);
    pf::free_plan_device(&p);
    p.opts = o;
    p.so = o.slope_order;
    p.c4 = 1.0 / (12.0 * std::log(p.beta));
    PF_HIP(hipGetDevice(&p.device));
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = o.dtype == PF_F64;
    p.sched = pf::default_schedule(p.n_phi, p.L, f64);
    rc = pf::build_tables_and_spectra(p, st);
    if (rc) {
        pf::free_plan_device(&p);
        return rc;
    }
    rc = pf::upload_twiddles(p.n_phi, f64, &p.twN);
    if (!rc) rc = pf::upload_twiddles(p.L, f64, &p.twL);
    if (!rc) {
        // forward: S (n_in rows) and the (Zr, Zp) pairs (n_r rows); transpose:
        // the (Vr, Vp) pairs and D (n_r rows each)
        // and after them the FP32 scale words (one set for the forward map,
        // one for the transpose; the notes are zero between calls)
        const size_t rows = std::max((size_t)p.n_in + 2 * (size_t)p.n_r, (size_t)3 * p.n_r);
        const size_t wsb = (rows * p.H * (f64 ? 16 : 8) + 255) / 256 * 256;
        hipError_t e = hipMalloc(&p.ws, wsb + 2 * pf::kScaleSet * sizeof(unsigned));
        if (e != hipSuccess) {
            pf::set_error("workspace allocation failed: %s", hipGetErrorString(e));
            rc = PF_ENOMEM;
        } else if (!f64) {
            p.gscale = (unsigned *)((unsigned char *)p.ws + wsb);
            e = hipMemsetAsync(p.gscale, 0, 2 * pf::kScaleSet * sizeof(unsigned), st);
            if (e != hipSuccess) {
                pf::set_error("hipMemsetAsync: %s", hipGetErrorString(e));
                rc = PF_EHIP;
            }
        }
    }
    if (!rc && p.wedges) rc = pf::build_wedge_spectra(p, st);
    if (rc) {
        pf::free_plan_device(&p);
        return rc;
    }
    if (!p.patch) rc = pf::autotune_plan(p, st);
    if (!rc) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            pf::set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
            rc = PF_EHIP;
        }
    }
    if (rc) {
        pf::free_plan_device(&p);
        return rc;
    }
    p.built = true;
    return PF_OK;
}

int pf_forces(pf_plan h, const void *sigma, void *f_r, void *f_phi, void *stream) {
    pf::clear_error();
    int rc = check_call(h, sigma, f_r, f_phi);
    if (rc) return rc;
    const Plan &p = h->p;
    if (p.wedges) {
        pf::set_error("the plan has origin wedges: call pf_forces_patches");
        return PF_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (p.opts.dtype == PF_F64)
        return forces_t<double>(p, (const double *)sigma, nullptr, (double *)f_r,
                                (double *)f_phi, st);
    return forces_t<float>(p, (const float *)sigma, nullptr, (float *)f_r, (float *)f_phi, st);
}

int pf_forces_patches(pf_plan h, const void *sigma_src, const void *sigma_wedge, void *f_r,
                      void *f_phi, void *stream) {
    pf::clear_error();
    int rc = check_call(h, sigma_src, f_r, f_phi);
    if (rc) return rc;
    const Plan &p = h->p;
    if (p.wedges != (sigma_wedge != nullptr)) {
        pf::set_error(p.wedges ? "the plan has origin wedges: sigma_wedge is required"
                               : "the plan has no origin wedges: sigma_wedge must be NULL");
        return PF_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (p.opts.dtype == PF_F64)
        return forces_t<double>(p, (const double *)sigma_src, (const double *)sigma_wedge,
                                (double *)f_r, (double *)f_phi, st);
    return forces_t<float>(p, (const float *)sigma_src, (const float *)sigma_wedge, (float *)f_r,
                           (float *)f_phi, st);
}

int pf_forces_backward(pf_plan h, const void *g_fr, const void *g_fphi, void *g_sigma,
                       void *stream) {
    pf::clear_error();
    int rc = check_call(h, g_fr, g_fphi, g_sigma);
    if (rc) return rc;
    const Plan &p = h->p;
    if (p.wedges) {
        pf::set_error("the plan has origin wedges: call pf_forces_patches_backward");
        return PF_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (p.opts.dtype == PF_F64)
        return backward_t<double>(p, (const double *)g_fr, (const double *)g_fphi,
                                  (double *)g_sigma, nullptr, st);
    return backward_t<float>(p, (const float *)g_fr, (const float *)g_fphi, (float *)g_sigma,
                             nullptr, st);
}

int pf_forces_patches_backward(pf_plan h, const void *g_fr, const void *g_fphi,
                               void *g_sigma_src, void *g_sigma_wedge, void *stream) {
    pf::clear_error();
    int rc = check_call(h, g_fr, g_fphi, g_sigma_src);
    if (rc) return rc;
    const Plan &p = h->p;
    if (p.wedges != (g_sigma_wedge != nullptr)) {
        pf::set_error(p.wedges ? "the plan has origin wedges: g_sigma_wedge is required"
                               : "the plan has no origin wedges: g_sigma_wedge must be NULL");
        return PF_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (p.opts.dtype == PF_F64)
        return backward_t<double>(p, (const double *)g_fr, (const double *)g_fphi,
                                  (double *)g_sigma_src, (double *)g_sigma_wedge, st);
    return backward_t<float>(p, (const float *)g_fr, (const float *)g_fphi,
                             (float *)g_sigma_src, (float *)g_sigma_wedge, st);
}

int pf_forces_timed(pf_plan h, int backward, const void *in0, const void *in1, void *out0,
                    void *out1, int reps, void *stream, float *pass_ms) {
    pf::clear_error();
    int rc = check_call(h, in0, out0, pass_ms);
    if (rc) return rc;
    if ((backward && !in1) || (!backward && !out1)) {
        pf::set_error("null field pointer");
        return PF_EINVAL;
    }
    if (reps < 1 || reps > 10000) {
        pf::set_error("reps = %d outside [1, 10000]", reps);
        return PF_EINVAL;
    }
    const Plan &p = h->p;
    if (p.patch && (backward || p.wedges)) {
        pf::set_error("timing of patch plans: forward without wedges only");
        return PF_EUNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k) {
        hipError_t e = hipEventCreate(&ev[k]);
        if (e != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
            pf::set_error("hipEventCreate: %s", hipGetErrorString(e));
            return PF_EHIP;
        }
    }
    rc = p.opts.dtype == PF_F64
             ? timed_t<double>(p, backward != 0, in0, in1, out0, out1, reps, st, ev)
             : timed_t<float>(p, backward != 0, in0, in1, out0, out1, reps, st, ev);
    if (!rc) {
        hipError_t e = hipEventSynchronize(ev[3]);
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            e = hipEventElapsedTime(&pass_ms[k], ev[k], ev[k + 1]);
            pass_ms[k] /= (float)reps;
        }
        if (e != hipSuccess) {
            pf::set_error("event timing: %s", hipGetErrorString(e));
            rc = PF_EHIP;
        }
    }
    for (int k = 0; k < 4; ++k) (void)hipEventDestroy(ev[k]);
    return rc;
}

}  // extern "C"

namespace {

// Arguments of a batched call: every plan built, single-grid, one precision,
// one device; ps[k] = the plans.
int check_batch(int n, const pf_plan *plans, const void *const *sigma, void *const *f_r,
                void *const *f_phi, const Plan **ps) {
    if (n < 1 || n > 4096 || !plans || !sigma || !f_r || !f_phi) {
        pf::set_error("bad batch arguments (n = %d)", n);
        return PF_EINVAL;
    }
    for (int k = 0; k < n; ++k) {
        int rc = check_call(plans[k], sigma[k], f_r[k], f_phi[k]);
        if (rc) return rc;
        ps[k] = &plans[k]->p;
        if (ps[k]->patch) {
            pf::set_error("batched plans must be single-grid plans (plan %d is a patch plan)", k);
            return PF_EUNSUPPORTED;
        }
        if (ps[k]->so != 2) {
            pf::set_error("batched plans must use slope order 2 (plan %d has %d)", k, ps[k]->so);
            return PF_EUNSUPPORTED;
        }
        if (ps[k]->opts.dtype != ps[0]->opts.dtype) {
            pf::set_error("batched plans must share one precision");
            return PF_EINVAL;
        }
        if (ps[k]->device != ps[0]->device) {
            pf::set_error("batched plans must live on one device");
            return PF_EINVAL;
        }
    }
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_forces_batched(int n, const pf_plan *plans, const void *const *sigma, void *const *f_r,
                      void *const *f_phi, void *stream) {
    pf::clear_error();
    std::vector<const Plan *> ps(n > 0 && n <= 4096 ? n : 0);
    int rc = check_batch(n, plans, sigma, f_r, f_phi, ps.data());
    if (rc) return rc;
    return pf::batched_forces(ps, sigma, f_r, f_phi, (hipStream_t)stream);
}

int pf_forces_batched_noalloc(int n, const pf_plan *plans, const void *const *sigma,
                              void *const *f_r, void *const *f_phi, void *stream) {
    pf::clear_error();
    const Plan *ps[256];
    if (n > 256) {
        pf::set_error("pf_forces_batched_noalloc takes at most 256 disks (got %d)", n);
        return PF_EINVAL;
    }
    int rc = check_batch(n, plans, sigma, f_r, f_phi, ps);
    if (rc) return rc;
    return pf::batched_forces_noalloc(ps, n, sigma, f_r, f_phi, (hipStream_t)stream);
}

}  // extern "C"
