// pf_common.hpp -- internal declarations shared by the libpf translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "fft_core.hpp"

namespace pf {

// thread-local error text behind pf_last_error()
void set_error(const char *fmt, ...);
void clear_error();

#define PF_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::pf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                  \
            return PF_EHIP;                                                       \
        }                                                                         \
    } while (0)

// Bytes allocated after the kernel spectra: the column passes copy each
// column's spectrum pairs into LDS in whole chunks of 64 lanes, which can
// reach up to L/E pairs past the column's last one; for the last column of
// the array those bytes are this tail, never used.
constexpr size_t kSpecTailPad = 64 * 1024;

// Launch shape of one transform pass: E points per thread and G transforms
// (rows or columns) per workgroup.
struct Shape {
    int E = 8;
    int G = 1;
};

// Schedule of a plan: launch shapes of the three passes for its sizes.
struct Schedule {
    Shape rows;       // one-channel row transforms along phi (forward pass A,
                      // transpose pass C; half-length M)
    Shape rows2;      // two-channel row transforms (forward pass C, transpose
                      // pass A)
    Shape cols;       // forward column pass along u (length L)
    Shape cols_adj;   // transpose column pass along u
};

struct Plan {
    // M = n_phi / 2; H = M stored columns of the packed half spectrum (column
    // 0 holds the real bins 0 and M); L = transform length along u; ldspec =
    // L / 2 + 1 stored k_u per spectrum column
    int n_r = 0, n_phi = 0, M = 0, H = 0, L = 0, ldspec = 0;
    // source rows s0 .. s0 + n_in - 1 of the grid (n_in = n_r, s0 = 0 for
    // one grid); n_r is the number of destination rows
    int n_in = 0, s0 = 0;
    bool patch = false;    // made by pf_plan_create_patches
    bool wedges = false;   // origin wedges [0, r_min beta^s0] below the source
    int col0 = 0;          // patch plans: source (and wedges) turned by col0 cells in phi
    double r_min = 0, r_max = 0, beta = 0, dphi = 0;
    // radial slope coefficients of g = r delta^r (three-point central, first
    // and last row); so = slope order of the build (2 or 4) and c4 the
    // five-point coefficient 1 / (12 ln beta)
    double ca = 0, c0 = 0, cn = 0;
    int so = 2;
    double c4 = 0;

    bool built = false;
    pf_build_opts opts{};
    int device = -1;
    double selfk[3] = {0, 0, 0};

    void *spec = nullptr;     // [2][H][ldspec] pairs (E', Q), plan precision
    void *twN = nullptr;      // n_phi-point twiddles, plan precision
    void *twL = nullptr;      // L-point twiddles, plan precision
    void *ws = nullptr;       // workspace: 3 * n_r * H complex, plan precision
                              // (forward: S, then (Zr, Zp) pairs; transpose:
                              // (Vr, Vp) pairs, then D)
    double *tables = nullptr; // [6][L][n_phi] FP64 (only with keep_tables)
    unsigned *gscale = nullptr; // FP32 scale words after the workspace: the
                                // forward map's set, then the transpose's
                                // (kScaleSet words each)
    void *wspec = nullptr;    // wedge spectra [2][n_r][H] pairs, plan precision
    void *wws = nullptr;      // wedge workspace: slope row, then its spectra
    Schedule sched;
    int64_t uid = 0;          // identity for batch-graph caching

    size_t elt() const { return opts.dtype == PF_F64 ? 8 : 4; }
};

// ---- kernels (pf_passes.hip) -----------------------------------------------
// Row transforms along phi of n_rows rows.  r2c: rows of in0 -> packed half
// spectra out ([n_rows][M] complex); with in1, rows of in0 and in1 -> pairs
// ([n_rows][M] pairs).  c2r: the inverse, from complex rows to out0, or from
// pairs to out0 and out1 when out1 is given.  g: the call's FP32 scale
// words (pass_bodies.hpp: r2c notes the largest magnitude in them, c2r
// clears them; nullptr: no scaling).  xin -> xout: one extra row of its own
// buffers in the same launch (one-channel transforms only; the origin
// wedges' row).
template <typename T>
int launch_rows_r2c(const Plan &p, const T *in0, const T *in1, int n_rows, cx<T> *out,
                    const cx<T> *twN, Shape s, hipStream_t st, unsigned *g = nullptr,
                    const T *xin = nullptr, cx<T> *xout = nullptr);
template <typename T>
int launch_rows_c2r(const Plan &p, const cx<T> *in, int n_rows, T *out0, T *out1,
                    const cx<T> *twN, Shape s, hipStream_t st, unsigned *g = nullptr,
                    int turn = 0, const cx<T> *xin = nullptr, T *xout = nullptr);
// Rows of n_phi = 2 Q P points, Q = 3 or 9, P a power of two (pf_rows3.hip):
// M = Q P.
template <typename T>
int launch_rows_r2cq(int M, const T *in0, const T *in1, int n_rows, cx<T> *out,
                     const cx<T> *twN, Shape s, hipStream_t st, unsigned *g, const T *xin,
                     cx<T> *xout);
template <typename T>
int launch_rows_c2rq(int M, const cx<T> *in, int n_rows, T *out0, T *out1, const cx<T> *twN,
                     Shape s, hipStream_t st, unsigned *g, int turn, const cx<T> *xin,
                     T *xout);
size_t rowsq_lds_bytes(int P, int Q, int G, int C, bool f64);
// The row transforms' M = n_phi / 2 complex points: a power of two, or
// three or nine times one (then Q sub-transforms of M / Q points);
// row_factor gives Q (1 for a power of two, 0 for other M), row_sub the
// points of one sub-transform, row_threads the threads per row at E points
// per thread.
inline bool is_pow2_int(int v) { return v > 0 && (v & (v - 1)) == 0; }
inline int row_factor(int M) {
    if (is_pow2_int(M)) return 1;
    if (M % 3 == 0 && is_pow2_int(M / 3)) return 3;
    if (M % 9 == 0 && is_pow2_int(M / 9)) return 9;
    return 0;
}
inline int row_sub(int M) { return row_factor(M) ? M / row_factor(M) : 0; }
inline int row_threads(int M, int E) { return row_sub(M) / E; }
// Column pass of the forward map (u-FFT, spectral multiply-accumulate with
// the spectral radial slope, inverse u-FFTs, crop): S ([n_in][H]) -> pairs
// Z ([n_r][H]); g: the scale words pass A noted (nullptr: unscaled).
template <typename T>
int launch_cols_fwd(const Plan &p, const cx<T> *S, cx<T> *Z, const cx<T> *spec,
                    const cx<T> *twL, Shape s, hipStream_t st, unsigned *g = nullptr);
// Column pass of the transpose: pairs V -> D.
template <typename T>
int launch_cols_adj(const Plan &p, const cx<T> *V, cx<T> *D, const cx<T> *spec,
                    const cx<T> *twL, Shape s, hipStream_t st, unsigned *g = nullptr);

// ---- kernels (pf_tables.hip) ------------------------------------------------
int build_tables_and_spectra(Plan &p, hipStream_t st);
// Origin-wedge spectra (plans with wedges) and the per-call wedge terms:
// Z += the wedges' contribution, from the wedge row's spectrum wrow (pass A
// transforms sigma_w into the plan's wedge workspace) and the first source
// row's spectrum S[0].
int build_wedge_spectra(Plan &p, hipStream_t st);
template <typename T>
int launch_wedge_terms(const Plan &p, const cx<T> *S, const cx<T> *wrow, cx<T> *Z,
                       hipStream_t st, const unsigned *g = nullptr);
// Transpose of the wedge terms (after the transpose's column pass, before
// its pass C): from the cotangents' row spectra V ((V_r, V_p) pairs on the
// n_r destination rows), the wedge row's spectrum into the plan's wedge
// workspace (pass C's launch transforms it into the wedge gradient), and the
// first source row's share of the wedges' radial slope added to D[0] (the
// source spectra pass C reads).
template <typename T>
int launch_wedge_adjoint_sums(const Plan &p, const cx<T> *V, cx<T> *D, hipStream_t st,
                              unsigned *g);

// ---- host helpers -------------------------------------------------------------
// exp(-2 pi i j / n) for j in [0, n), computed in long double
void twiddles_host(int n, std::vector<double> &re, std::vector<double> &im);
int upload_twiddles(int n, bool f64, void **dst);
Schedule default_schedule(int n_phi, int L, bool f64);
bool valid_shape_rows(int M, Shape s, bool f64);
bool valid_shape_cols(int L, Shape s, bool f64);
// LDS bytes of a column-pass workgroup: the transform buffers and, with the
// prefetch, the spectrum region
size_t cols_lds_bytes(int L, int E, int G, bool f64, bool prefetch);

inline int ilog2(int v) {
    int k = 0;
    while ((1 << k) < v) ++k;
    return k;
}

}  // namespace pf
