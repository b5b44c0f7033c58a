// pf_cart.hip -- the Cartesian second-order method and the Cartesian
// particle and modified particle methods (Sec. 3.1, Eq. 6-21, A1-A16) on a
// uniform N_x x N_y grid, as a 2-D convolution on the GPU with the same
// three-pass structure as the log-polar path, zero-padded in both directions
// (L_x >= 2 N_x, L_y >= 2 N_y: the circular convolution equals the linear
// one on the grid, so no artificial boundary enters):
//
//   pass A  rows (index i along x): the y-slope delta^y is formed in the row
//           (central differences, one-sided on the first and last cells),
//           then (S, Dy) = R2C_y(sigma, delta^y), pairs [N_x][H], H = L_y/2
//   pass B  per column k_y:  X = FFT_x(pad S[:, k_y]),  D = FFT_x(pad Dy[:, k_y])
//             Zx = IFFT_x(E'_x X + Q_x B(S) + R_x D)
//             Zy = IFFT_x(E'_y X + Q_y B(S) + R_y D),      pairs [N_x][H]
//   pass C  F^x = C2R_y(Zx), F^y = C2R_y(Zy), the first N_y points of each row
//
// with the kernel spectra (2-D transforms of the tables of Eq. 13-15 and
// A5-A7, zero-padded and wrapped, scaled by 1 / (L_x L_y))
//   E'_x = K^{x,0} + D_x K^{x,x},  Q_x = K^{x,x},  R_x = K^{x,y}
//   E'_y = K^{y,0} + D_x K^{y,x},  Q_y = K^{y,x},  R_y = K^{y,y}
// where D_x = 2i ca sin(2 pi k_x / L_x) is the transform of the central
// difference in x on the zero-padded column and B(S) the transform of its
// four-row correction (the same device as the log-polar radial slope, with
// ca = 1 / (2 Delta x) and one-sided first and last rows, c0 = cn =
// 1 / Delta x).
//
// Parity in the y offset n: K^{x,0}, K^{x,x}, K^{y,y} are even, K^{x,y},
// K^{y,0}, K^{y,x} odd; so (E'_x, Q_x) and R_y mirror as the conjugate in
// k_x, (E'_y, Q_y) and R_x as minus the conjugate, and only k_x in
// [0, L_x/2] is stored.  Column 0 of the packed half spectrum carries the
// real bins 0 and L_y/2 together; the odd spectra vanish there, so its
// slots hold: pair 0 = (E'_x, Q_x) of bin 0, pair 1 = (E'_x, Q_x) of bin
// L_y/2, R slot 0 = R_y of bin L_y/2, R slot 1 = R_y of bin 0.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "pass_bodies.hpp"
#include "pf_common.hpp"

namespace pf {
namespace {

// ---------------------------------------------------------------------------
// Cell kernels of the second-order method (Eq. 13-15, A5-A7) for the source
// cell whose centre is (X, Y) relative to the destination: the closed forms
// A8-A13 near the destination, where they are accurate; farther away the
// same integrals by a 16 x 16 Gauss-Legendre rule (the closed double
// differences lose digits to cancellation there; the rule's error falls
// like (h / 2d)^32, below 1e-24 from three cell sizes on).
// Output order: K^{x,0}, K^{x,x}, K^{x,y}, K^{y,0}, K^{y,y}, K^{y,x}.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cart_ln(double y, double x, double rho) {
    // ln(y + sqrt(x^2 + y^2)), rationalised for y < 0
    return y >= 0.0 ? log(y + rho) : log(x * x / (rho - y));
}

__device__ void cart_cell(double X, double Y, double dx, double dy,
                          const double *__restrict__ gl, double K[6]) {
    const double d = sqrt(X * X + Y * Y);
    if (d < 3.0 * fmax(dx, dy)) {
        const double xs[2] = {X - 0.5 * dx, X + 0.5 * dx};
        const double ys[2] = {Y - 0.5 * dy, Y + 0.5 * dy};
        double ly = 0, lx = 0, ylx = 0, xly = 0, rr = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const double sg = (a == b) ? 1.0 : -1.0;   // f|^{x_u}_{x_l}|^{y_u}_{y_l}
                const double x = xs[a], y = ys[b];
                const double rho = sqrt(x * x + y * y);
                const double Ly = cart_ln(y, x, rho), Lx = cart_ln(x, y, rho);
                ly += sg * Ly;
                lx += sg * Lx;
                ylx += sg * y * Lx;
                xly += sg * x * Ly;
                rr += sg * rho;
            }
        const double kx0 = -ly, ky0 = -lx;
        K[0] = kx0;
        K[1] = -X * kx0 + ylx;   // (x_i - x_i') K^{x,0} + ...
        K[2] = -Y * kx0 - rr;
        K[3] = ky0;
        K[4] = -Y * ky0 + xly;
        K[5] = -X * ky0 - rr;
        return;
    }
    // gl: 16 nodes then 16 weights on [-1, 1]
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int p = 0; p < 16; ++p) {
        const double u = 0.5 * dx * gl[p];      // xbar - x_i'
        const double x = X + u;                  // xbar - x_i
        double b[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const double v = 0.5 * dy * gl[q];   // ybar - y_j'
            const double y = Y + v;
            const double r2 = x * x + y * y;
            const double w = gl[16 + q] / (r2 * sqrt(r2));
            b[0] += w * x;
            b[1] += w * x * u;
            b[2] += w * x * v;
            b[3] += w * y;
            b[4] += w * y * v;
            b[5] += w * y * u;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k] += gl[16 + p] * b[k];
    }
    const double jac = 0.25 * dx * dy;
#pragma unroll
    for (int k = 0; k < 6; ++k) K[k] = a[k] * jac;
}

struct CartGeo {
    int n_x, n_y, Lx, Ly, method;
    double dx, dy;
};

// The six tables on the zero-padded, wrapped L_x x L_y grid, FP64, layout
// [6][L_x][L_y]: entry (a, b) holds the offset m = a (or a - L_x), n = b (or
// b - L_y) when |m| < N_x and |n| < N_y, zero otherwise.  method 0: the
// second-order kernels; 1: the particle kernel (Eq. 20, A15) with masses
// sigma Dx Dy and no self force; 2: that plus K^{x,x}_{00} and K^{y,y}_{00}
// in the (0, 0) entries (Eq. 21, A16; the other self terms vanish by
// symmetry).
__global__ __launch_bounds__(256) void k_cart_tables(CartGeo g, const double *__restrict__ gl,
                                                     double *__restrict__ tab) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (b >= g.Ly) return;
    const int m = a < g.Lx / 2 ? a : a - g.Lx;
    const int n = b < g.Ly / 2 ? b : b - g.Ly;
    double K[6] = {0, 0, 0, 0, 0, 0};
    if (abs(m) < g.n_x && abs(n) < g.n_y) {
        const double X = -m * g.dx, Y = -n * g.dy;   // source centre - destination
        if (g.method == 0) {
            cart_cell(X, Y, g.dx, g.dy, gl, K);
        } else if (m != 0 || n != 0) {
            const double d2 = X * X + Y * Y;
            const double w = g.dx * g.dy / (d2 * sqrt(d2));
            K[0] = w * X;
            K[3] = w * Y;
        } else if (g.method == 2) {
            double S[6];
            cart_cell(0.0, 0.0, g.dx, g.dy, gl, S);
            K[1] = S[1];
            K[4] = S[4];
        }
    }
    const size_t plane = (size_t)g.Lx * g.Ly;
#pragma unroll
    for (int k = 0; k < 6; ++k) tab[k * plane + (size_t)a * g.Ly + b] = K[k];
}

// Spectra from the row spectra of the tables (rowspec [6][L_x][H] complex,
// packed half spectrum along y): per column k_y (block kb in [0, H]; kb = H
// is bin L_y/2, taken from the imaginary part of column 0) the six
// transforms along x, combined as in the header and stored for
// k_x in [0, L_x/2].
template <int L, int E>
__global__ __launch_bounds__(512) void k_cart_fold(const cx<double> *__restrict__ rowspec, int H,
                                                   double ca, double sc,
                                                   cx2<double> *__restrict__ spec,
                                                   cx<double> *__restrict__ rsp, int ldspec,
                                                   const cx<double> *__restrict__ twL) {
    constexpr int TH = L / E;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double> *buf = reinterpret_cast<cx<double> *>(smem_raw);
    const int kb = blockIdx.x, t = threadIdx.x;
    const int src = kb == H ? 0 : kb;
    const int part = kb == 0 ? 1 : (kb == H ? 2 : 0);   // 1: bin 0, 2: bin L_y/2
    Lds<double> lds{buf, 0, 1};
    Twiddles<L, E, double> tw;
    tw.load(t, twL, 1);

    auto load = [&](int tab, cx<double>(&v)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = t + e * TH;
            cx<double> x = rowspec[((size_t)tab * L + row) * H + src];
            if (part == 1) x = cx<double>{x.x, 0.0};
            if (part == 2) x = cx<double>{x.y, 0.0};
            v[e] = x;
        }
        fft_fwd<L, E, double>(v, t, lds, tw);
    };
    auto store_pair = [&](int slot, const cx<double>(&a)[E], const cx<double>(&q)[E]) {
        cx2<double> *dst = spec + ((size_t)slot * H + src) * ldspec;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ku = t + e * TH;
            if (ku <= L / 2) dst[ku] = cx2<double>{a[e], q[e]};
        }
    };
    auto store_r = [&](int slot, const cx<double>(&a)[E]) {
        cx<double> *dst = rsp + ((size_t)slot * H + src) * ldspec;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ku = t + e * TH;
            if (ku <= L / 2) dst[ku] = scale(a[e], sc);
        }
    };
    // (E', Q) of one output from its density table t0 and x-slope table ts
    auto pair = [&](int t0, int ts, int slot) {
        cx<double> a[E], q[E];
        load(ts, q);
        load(t0, a);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ku = t + e * TH;
            const double d = 2.0 * ca * sinpi(2.0 * ku / L);
            const cx<double> qe = scale(q[e], sc), ae = scale(a[e], sc);
            a[e] = cx<double>{ae.x - d * qe.y, ae.y + d * qe.x};   // K0 + i d Ks
            q[e] = qe;
        }
        store_pair(slot, a, q);
    };
    cx<double> r[E];
    if (part == 0) {
        pair(0, 1, 0);   // F^x: K^{x,0}, K^{x,x}
        pair(3, 5, 1);   // F^y: K^{y,0}, K^{y,x}
        load(2, r);      // K^{x,y}
        store_r(0, r);
        load(4, r);      // K^{y,y}
        store_r(1, r);
    } else {
        pair(0, 1, part == 1 ? 0 : 1);
        load(4, r);
        store_r(part == 1 ? 1 : 0, r);
    }
}

__global__ void k_cart_to_f32(const double *__restrict__ in, float *__restrict__ out, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// Pass A: G rows (blocked) x (M/E) threads; LDS 2 G padded_len(M) complex.
// A real row of L_y = 2M points (sigma and delta^y, zero beyond N_y) goes
// through one M-point complex transform of z[k] = x[2k] + i x[2k+1] per
// channel; points k >= M/2 are padding (2k >= M >= N_y), so the first stage
// skips them.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T cart_dy(int j, int n_y, T l, T c, T r, T idy) {
    if (j >= n_y) return T(0);
    if (j == 0) return (r - c) * idy;
    if (j == n_y - 1) return (c - l) * idy;
    return (r - l) * (T(0.5) * idy);
}

// gscale: the FP32 grid scale's words (pass_bodies.hpp), as in the polar
// passes: pass A notes the largest magnitude of its rows (sigma and its
// y-slope), pass B scales its columns by 2^-e after the first transform
// stage, pass C restores 2^e and clears the notes; nullptr in FP64.
template <typename T, int M, int E>
__device__ __forceinline__ void body_cart_rows(int unit, int G, cx<T> *__restrict__ buf,
                                               const T *__restrict__ sigma, int n_x, int n_y,
                                               T idy, cx2<T> *__restrict__ out,
                                               const cx<T> *__restrict__ twN,
                                               unsigned *__restrict__ gscale) {
    constexpr int TH = M / E;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_x;
    const int i = active ? row : 0;
    Lds<T> lds[2];
    row_lds<T, M, E, 2>(buf, gi, G, lds);
    const T *s = sigma + (size_t)i * n_y;
    // neighbour values, zero outside the row; the load itself is always in bounds
    auto at = [&](int j) -> T {
        const T val = s[j < 0 ? 0 : (j >= n_y ? n_y - 1 : j)];
        return (j >= 0 && j < n_y) ? val : T(0);
    };

    cx<T> v[2][E];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int j0 = 2 * (t + e * TH);
        const T am = at(j0 - 1), a0 = at(j0), a1 = at(j0 + 1), a2 = at(j0 + 2);
        v[0][e] = cx<T>{a0, a1};
        v[1][e] = cx<T>{cart_dy(j0, n_y, am, a0, a1, idy), cart_dy(j0 + 1, n_y, a0, a1, a2, idy)};
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e >= E / 2 || !active) v[c][e] = cx<T>{T(0), T(0)};
    scale_note<T, E, 2>(gscale, v);
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
    fft_fwd<M, E, 2, T, true>(v, t, lds, tw);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[c].st_split(lds_pad(t), e * TH, v[c][e]);
    __syncthreads();
    cx<T> o[2][E];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            const cx<T> zk = lds[c].ld(k), zm = lds[c].ld((M - k) & (M - 1));
            const cx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            const cx<T> od = {T(0.5) * (zk.y + zm.y), -T(0.5) * (zk.x - zm.x)};
            cx<T> x = ev + cmul(twN[k], od);
            if (k == 0) x = cx<T>{zk.x + zk.y, zk.x - zk.y};   // (X_0, X_M), both real
            o[c][e] = x;
        }
    if (active) {
        cx2<T> *orow = out + (size_t)i * M;
#pragma unroll
        for (int e = 0; e < E; ++e) store_stream(&orow[t + e * TH], cx2<T>{o[0][e], o[1][e]});
    }
}

// Pass C: pairs [N_x][M] -> the first N_y points of the real rows of f_x, f_y.
template <typename T, int M, int E>
__device__ __forceinline__ void body_cart_c2r(int unit, int G, cx<T> *__restrict__ buf,
                                              const cx2<T> *__restrict__ in, int n_x, int n_y,
                                              T *__restrict__ out0, T *__restrict__ out1,
                                              const cx<T> *__restrict__ twN,
                                              unsigned *__restrict__ gscale) {
    constexpr int TH = M / E;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_x;
    const int i = active ? row : 0;
    Lds<T> lds[2];
    row_lds<T, M, E, 2>(buf, gi, G, lds);

    // the thread's bins k from global memory, the mirror bins M - k from LDS
    cx<T> xk[2][E], xm[2][E], wk[E];
    const cx2<T> *X = in + (size_t)i * M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
        const cx2<T> a = X[k];
        xk[0][e] = a.a;
        xk[1][e] = a.b;
        wk[e] = twN[k];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[c].st_split(lds_pad(t), e * TH, xk[c][e]);
    lds_barrier();
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) xm[c][e] = lds[c].ld((M - (t + e * TH)) & (M - 1));
    lds_barrier();
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
    if (t == 0) {   // unpack bin 0 = (X_0, X_M)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const cx<T> p = xk[c][0];
            xk[c][0] = cx<T>{p.x, T(0)};
            xm[c][0] = cx<T>{p.y, T(0)};
        }
    }
    cx<T> v[2][E];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cx<T> s = {xk[c][e].x + xm[c][e].x, xk[c][e].y - xm[c][e].y};
            const cx<T> d = {xk[c][e].x - xm[c][e].x, xk[c][e].y + xm[c][e].y};
            const cx<T> dw = cmulc(d, wk[e]);
            v[c][e] = active ? cx<T>{s.x - dw.y, s.y + dw.x} : cx<T>{T(0), T(0)};
        }
    fft_inv<M, E, 2, T>(v, t, lds, tw);
    const T up = scale_finish<T>(gscale, unit);
    if (up != T(1))
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int e = 0; e < E; ++e) v[c][e] = scale(v[c][e], up);
    if (active) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T *o = (c == 0 ? out0 : out1) + (size_t)i * n_y;
            // points e >= E/2 hold y >= M >= N_y: never stored
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                const int j = 2 * (t + e * TH);
                // streaming stores, as in the polar row passes
                if (j < n_y) __builtin_nontemporal_store(v[c][e].x, &o[j]);
                if (j + 1 < n_y) __builtin_nontemporal_store(v[c][e].y, &o[j + 1]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass B: G columns (interleaved lane by lane) x (L/E) threads; LDS two
// regions of G padded_len(L) complex.
// ---------------------------------------------------------------------------
// PF: the pairs (E'_x, Q_x) go to LDS at spl (G spec_prefetch_len<L, E>()
// pairs, an LDS array of its own) while the two columns are transformed.
template <typename T, int L, int E, bool PF = false>
__device__ __forceinline__ void body_cart_cols(int unit, int G, cx<T> *__restrict__ buf,
                                               const cx2<T> *__restrict__ SD,
                                               cx2<T> *__restrict__ Z,
                                               const cx2<T> *__restrict__ spec,
                                               const cx<T> *__restrict__ rsp, int H, int n_x,
                                               int ldspec, T ca, T c0, T cn,
                                               const cx<T> *__restrict__ twL,
                                               cx2<T> *spl = nullptr,
                                               unsigned *__restrict__ gscale = nullptr) {
    constexpr int TH = L / E;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = unit * G + gi;
    const bool valid = col < H;
    const int cl = valid ? col : 0;
    const bool packed = unit == 0;
    const bool is0 = packed && gi == 0;
    const Lds<T> lS{buf, gi, G};
    const Lds<T> lD{buf + (size_t)G * padded_len(L), gi, G};

    // the scale note first (loads complete in order)
    const unsigned note = scale_load<T>(gscale);
    cx<T> v[2][E];   // v[0]: S column, v[1]: Dy column
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int i = t + e * TH;
        const cx2<T> q = SD[(size_t)(i < n_x ? i : n_x - 1) * H + cl];
        v[0][e] = q.a;
        v[1][e] = q.b;
    }
    const cx<T> x0 = SD[cl].a, x1 = SD[(size_t)H + cl].a;
    const cx<T> xm2 = SD[(size_t)(n_x - 2) * H + cl].a, xm1 = SD[(size_t)(n_x - 1) * H + cl].a;
    const cx<T> wt = twL[t], wnt = twL[(int)(((unsigned)n_x * (unsigned)t) & (unsigned)(L - 1))];
    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
    // issued after the column's loads, which the transforms wait for
    if constexpr (PF) prefetch_spectra<T, L, E>(unit, G, H, ldspec, spec, spl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (e >= E / 2 || !valid || i >= n_x) {
            v[0][e] = cx<T>{T(0), T(0)};
            v[1][e] = cx<T>{T(0), T(0)};
        }
    }
    GridScale<T> sc;
    fft_col_fwd<L, E, T>(v[0], t, lS, tw, ScaleFind<T>{gscale, note, unit, &sc});
    fft_col_fwd<L, E, T>(v[1], t, lD, tw, ScaleKnown<T>{sc.dn});
    if (packed) {   // column 0 reads the conjugate mirror points from LDS
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lS.st_split(lds_pad(t), e * TH, v[0][e]);
            lD.st_split(lds_pad(t), e * TH, v[1][e]);
        }
        lds_barrier();
    }
    const cx2<T> *s0l = PF ? spl + (size_t)gi * spec_prefetch_len<L, E>() : nullptr;
    if constexpr (PF) {
        // the prefetch has landed for this wave; the barrier makes every
        // wave's chunks visible
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    const cx2<T> *s0 = spec + (size_t)cl * ldspec;          // (E'_x, Q_x)
    const cx2<T> *s1 = spec + (size_t)(H + cl) * ldspec;    // (E'_y, Q_y)
    const cx<T> *r0 = rsp + (size_t)cl * ldspec;            // R_x
    const cx<T> *r1 = rsp + (size_t)(H + cl) * ldspec;      // R_y
    const SlopeFix<T> a = slope_fix(scale(x0, sc.dn), scale(x1, sc.dn), scale(xm2, sc.dn),
                                    scale(xm1, sc.dn), ca, c0, cn);
    const SlopePhasors<T> ph = slope_phasors(a, wt, wnt);
    SlopePhasors<T> ph0 = ph, phM = ph;
    if (is0) {
        ph0 = slope_phasors(slope_fix_part(a, false), wt, wnt);
        phM = slope_phasors(slope_fix_part(a, true), wt, wnt);
    }
    // spectrum loads per batch: six complex values per point
    constexpr int CH = sizeof(T) == 8 ? 1 : 4;
    const bool t0 = t == 0;
#pragma unroll
    for (int cb = 0; cb < E; cb += CH) {
        cx2<T> pa[CH], pb[CH];
        cx<T> ra[CH], rb[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int ix = spec_index<L, E>(t, cb + j);
            pa[j] = PF ? s0l[ix] : s0[ix];
            pb[j] = s1[ix];
            ra[j] = r0[ix];
            rb[j] = r1[ix];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = cb + j;
            const cx<T> rne = root_ne<T, L, E>(twL, n_x, e);
            cx<T> y0, y1;
            if (is0) {
                const int mk = (L - (t + e * TH)) & (L - 1);
                const cx<T> mS = lS.ld(mk), mD = lD.ld(mk);
                const cx<T> AS = unpack_even(v[0][e], mS), BS = unpack_odd(v[0][e], mS);
                const cx<T> AD = unpack_even(v[1][e], mD), BD = unpack_odd(v[1][e], mD);
                const cx<T> f0 = slope_fix_at<T, E>(ph0, rne, e);
                const cx<T> fM = slope_fix_at<T, E>(phM, rne, e);
                const cx<T> zx0 = spec_mac<T, E, false, false>(
                    spec_mul<T, E, false, false>(pa[j].a, AS, e, t0), pa[j].b, f0, e, t0);
                const cx<T> zxM = spec_mac<T, E, false, false>(
                    spec_mul<T, E, false, false>(pb[j].a, BS, e, t0), pb[j].b, fM, e, t0);
                const cx<T> zy0 = spec_mul<T, E, false, false>(rb[j], AD, e, t0);
                const cx<T> zyM = spec_mul<T, E, false, false>(ra[j], BD, e, t0);
                y0 = cx<T>{zx0.x - zxM.y, zx0.y + zxM.x};   // bin 0 + i bin M
                y1 = cx<T>{zy0.x - zyM.y, zy0.y + zyM.x};
            } else {
                const cx<T> f = slope_fix_at<T, E>(ph, rne, e);
                y0 = spec_mac<T, E, true, false>(
                    spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pa[j].a, v[0][e], e, t0), pa[j].b, f, e, t0),
                    ra[j], v[1][e], e, t0);
                y1 = spec_mac<T, E, false, false>(
                    spec_mac<T, E, true, false>(
                        spec_mul<T, E, true, false>(pb[j].a, v[0][e], e, t0), pb[j].b, f, e, t0),
                    rb[j], v[1][e], e, t0);
            }
            v[0][e] = y0;
            v[1][e] = y1;
        }
    }
    if (packed) lds_barrier();
    fft_inv<L, E, T>(v[0], t, lS, tw);
    fft_inv<L, E, T>(v[1], t, lD, tw);
    if (valid) {
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {   // rows lie in the first half (L >= 2 N_x)
            const int i = t + e * TH;
            if (i < n_x) Z[(size_t)i * H + col] = cx2<T>{v[0][e], v[1][e]};
        }
    }
}

__device__ __forceinline__ int cart_xcd_group(int b, int per_xcd) {
    return (b & 7) * per_xcd + (b >> 3);
}

template <typename T, int M, int E>
__global__ __launch_bounds__(512) void k_cart_rows(const T *__restrict__ sigma, int n_x, int n_y,
                                                   T idy, cx2<T> *__restrict__ out,
                                                   const cx<T> *__restrict__ twN,
                                                   unsigned *__restrict__ gscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    body_cart_rows<T, M, E>(blockIdx.x, blockDim.x / (M / E), reinterpret_cast<cx<T> *>(smem_raw),
                            sigma, n_x, n_y, idy, out, twN, gscale);
}

template <typename T, int M, int E>
__global__ __launch_bounds__(512) void k_cart_c2r(const cx2<T> *__restrict__ in, int n_x,
                                                  int n_y, T *__restrict__ out0,
                                                  T *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN,
                                                  unsigned *__restrict__ gscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    body_cart_c2r<T, M, E>(blockIdx.x, blockDim.x / (M / E), reinterpret_cast<cx<T> *>(smem_raw),
                           in, n_x, n_y, out0, out1, twN, gscale);
}

template <typename T, int L, int E>
__global__ __launch_bounds__(512) void k_cart_cols(const cx2<T> *__restrict__ SD,
                                                   cx2<T> *__restrict__ Z,
                                                   const cx2<T> *__restrict__ spec,
                                                   const cx<T> *__restrict__ rsp, int H, int n_x,
                                                   int ldspec, T ca, T c0, T cn,
                                                   const cx<T> *__restrict__ twL, int per_xcd,
                                                   int n_groups, unsigned *__restrict__ gscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int grp = cart_xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;   // whole workgroup leaves together
    body_cart_cols<T, L, E>(grp, blockDim.x / (L / E), reinterpret_cast<cx<T> *>(smem_raw), SD,
                            Z, spec, rsp, H, n_x, ldspec, ca, c0, cn, twL, nullptr, gscale);
}

// Column workgroup size of the Cartesian pass: one column of L / E threads,
// or 256 / (L / E) columns when a column has fewer than 256 threads.
__host__ __device__ constexpr int cart_cols_g(int L, int E) {
    return L / E >= 256 ? 1 : 256 / (L / E);
}

// The static LDS of the prefetching column kernel (two transform buffers
// and the prefetch region); it is used when that fits two workgroups per CU.
template <typename T, int L, int E>
constexpr size_t cart_cols_pf_lds() {
    constexpr int G = cart_cols_g(L, E);
    return (size_t)2 * G * padded_len(L) * sizeof(cx<T>) +
           (size_t)G * spec_prefetch_len<L, E>() * sizeof(cx2<T>);
}

template <typename T, int L, int E>
__global__ __launch_bounds__(512) void k_cart_cols_pf(const cx2<T> *__restrict__ SD,
                                                      cx2<T> *__restrict__ Z,
                                                      const cx2<T> *__restrict__ spec,
                                                      const cx<T> *__restrict__ rsp, int H,
                                                      int n_x, int ldspec, T ca, T c0, T cn,
                                                      const cx<T> *__restrict__ twL, int per_xcd,
                                                      int n_groups, unsigned *__restrict__ gscale) {
    constexpr int G = cart_cols_g(L, E);
    __shared__ cx<T> fbuf[2 * G * padded_len(L)];
    __shared__ cx2<T> spl[G * spec_prefetch_len<L, E>()];
    const int grp = cart_xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;   // whole workgroup leaves together
    body_cart_cols<T, L, E, true>(grp, G, fbuf, SD, Z, spec, rsp, H, n_x, ldspec, ca, c0, cn, twL,
                                  spl, gscale);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct CartPlan {
    int n_x = 0, n_y = 0, Lx = 0, Ly = 0, H = 0, ldspec = 0;
    double dx = 0, dy = 0;
    int dtype = PF_F32, method = PF_CART_SECOND;
    bool built = false;
    void *spec = nullptr;   // [2][H][ldspec] pairs (E', Q), plan precision
    void *rsp = nullptr;    // [2][H][ldspec] complex R, plan precision
    void *twN = nullptr;    // L_y-point twiddles
    void *twL = nullptr;    // L_x-point twiddles
    void *ws = nullptr;     // (S, Dy) pairs then (Zx, Zy) pairs, 2 N_x H each, then
                            // (FP32) the grid scale's words
    unsigned *gscale = nullptr;
    Shape rows, cols;
};

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

void free_cart(CartPlan &c) {
    for (void **q : {&c.spec, &c.rsp, &c.twN, &c.twL, &c.ws}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    c.gscale = nullptr;   // inside ws
    c.built = false;
}

// n-point Gauss-Legendre nodes and weights on [-1, 1] by Newton's iteration
// on the Legendre polynomial (three-term recurrence), in long double.
void gauss_legendre_host(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            const long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {   // derivative at the converged node
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
        }
        const long double wt = 2 / ((1 - z * z) * dp * dp);
        x[i] = (double)(-z);
        x[n - 1 - i] = (double)z;
        w[i] = w[n - 1 - i] = (double)wt;
    }
}

Shape cart_rows_shape(int M) {
    Shape s;
    s.E = M >= 2048 ? 16 : (M < 8 ? M : 8);
    const int th = M / s.E;
    s.G = th >= 128 ? 1 : 128 / th;
    return s;
}

// The column body holds two transforms and six spectra per point: E = 8
// points per thread in FP32 and 4 in FP64 keep it within the register file
// (it spills at 16 and 8 respectively); FP64 at L = 4096 takes E = 8 to stay
// within 512 threads per column.
__host__ __device__ constexpr int cart_cols_e(int L, bool f64) { return f64 && L < 4096 ? 4 : 8; }

Shape cart_cols_shape(int L, bool f64) {
    Shape s;
    s.E = cart_cols_e(L, f64);
    s.G = cart_cols_g(L, s.E);
    return s;
}

template <typename K>
int allow_lds_cart(K kern, size_t lds) {
    if (lds > 64 * 1024)
        PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PF_OK;
}

template <typename T, int M>
int rows_m(const CartPlan &c, bool pass_c, const void *in, void *o0, void *o1, hipStream_t st) {
    constexpr int E = M >= 2048 ? 16 : (M < 8 ? M : 8);
    const Shape s = cart_rows_shape(M);
    const int blocks = (c.n_x + s.G - 1) / s.G;
    const size_t lds = (size_t)2 * s.G * padded_len(M) * sizeof(cx<T>);
    const cx<T> *tw = (const cx<T> *)c.twN;
    if (!pass_c) {
        int rc = allow_lds_cart(k_cart_rows<T, M, E>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL((k_cart_rows<T, M, E>), dim3(blocks), dim3(s.G * (M / E)), lds, st,
                           (const T *)in, c.n_x, c.n_y, T(1.0 / c.dy), (cx2<T> *)o0, tw,
                           sizeof(T) == 4 ? c.gscale : nullptr);
    } else {
        int rc = allow_lds_cart(k_cart_c2r<T, M, E>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL((k_cart_c2r<T, M, E>), dim3(blocks), dim3(s.G * (M / E)), lds, st,
                           (const cx2<T> *)in, c.n_x, c.n_y, (T *)o0, (T *)o1, tw,
                           sizeof(T) == 4 ? c.gscale : nullptr);
    }
    PF_HIP(hipGetLastError());
    return PF_OK;
}

template <typename T>
int launch_cart_rows(const CartPlan &c, bool pass_c, const void *in, void *o0, void *o1,
                     hipStream_t st) {
    switch (c.H) {
        case 4: return rows_m<T, 4>(c, pass_c, in, o0, o1, st);
        case 8: return rows_m<T, 8>(c, pass_c, in, o0, o1, st);
        case 16: return rows_m<T, 16>(c, pass_c, in, o0, o1, st);
        case 32: return rows_m<T, 32>(c, pass_c, in, o0, o1, st);
        case 64: return rows_m<T, 64>(c, pass_c, in, o0, o1, st);
        case 128: return rows_m<T, 128>(c, pass_c, in, o0, o1, st);
        case 256: return rows_m<T, 256>(c, pass_c, in, o0, o1, st);
        case 512: return rows_m<T, 512>(c, pass_c, in, o0, o1, st);
        case 1024: return rows_m<T, 1024>(c, pass_c, in, o0, o1, st);
        case 2048: return rows_m<T, 2048>(c, pass_c, in, o0, o1, st);
    }
    set_error("Cartesian row transform of %d points not built", 2 * c.H);
    return PF_EUNSUPPORTED;
}

template <typename T, int L>
int cols_l(const CartPlan &c, const void *SD, void *Z, hipStream_t st) {
    constexpr int E = cart_cols_e(L, sizeof(T) == 8);
    const Shape s = cart_cols_shape(L, sizeof(T) == 8);
    const int n_groups = (c.H + s.G - 1) / s.G;
    const int per_xcd = (n_groups + 7) / 8;
    // The (E'_x, Q_x) prefetch where its LDS keeps the occupancy the
    // registers allow: FP32 within 80 KB (two workgroups per CU), and any
    // column of 512 threads (one workgroup per CU either way) within 144 KB.
    constexpr size_t kPfLds = L / E >= 512 ? 144 * 1024 : (sizeof(T) == 4 ? 80 * 1024 : 0);
    if constexpr (L / E >= 64 && cart_cols_pf_lds<T, L, E>() <= kPfLds) {
        // 32-bit offsets over that half
        if ((size_t)c.H * c.ldspec * sizeof(cx2<T>) >= ((size_t)1 << 31)) {
            set_error("Cartesian spectra too large for the column pass prefetch");
            return PF_EUNSUPPORTED;
        }
        hipLaunchKernelGGL((k_cart_cols_pf<T, L, E>), dim3(per_xcd * 8), dim3(s.G * (L / E)), 0,
                           st, (const cx2<T> *)SD, (cx2<T> *)Z, (const cx2<T> *)c.spec,
                           (const cx<T> *)c.rsp, c.H, c.n_x, c.ldspec, T(0.5 / c.dx),
                           T(1.0 / c.dx), T(1.0 / c.dx), (const cx<T> *)c.twL, per_xcd, n_groups,
                           sizeof(T) == 4 ? c.gscale : nullptr);
        PF_HIP(hipGetLastError());
        return PF_OK;
    }
    const size_t lds = (size_t)2 * s.G * padded_len(L) * sizeof(cx<T>);
    int rc = allow_lds_cart(k_cart_cols<T, L, E>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_cart_cols<T, L, E>), dim3(per_xcd * 8), dim3(s.G * (L / E)), lds, st,
                       (const cx2<T> *)SD, (cx2<T> *)Z, (const cx2<T> *)c.spec,
                       (const cx<T> *)c.rsp, c.H, c.n_x, c.ldspec, T(0.5 / c.dx), T(1.0 / c.dx),
                       T(1.0 / c.dx), (const cx<T> *)c.twL, per_xcd, n_groups,
                       sizeof(T) == 4 ? c.gscale : nullptr);
    PF_HIP(hipGetLastError());
    return PF_OK;
}

template <typename T>
int launch_cart_cols(const CartPlan &c, const void *SD, void *Z, hipStream_t st) {
    switch (c.Lx) {
        case 8: return cols_l<T, 8>(c, SD, Z, st);
        case 16: return cols_l<T, 16>(c, SD, Z, st);
        case 32: return cols_l<T, 32>(c, SD, Z, st);
        case 64: return cols_l<T, 64>(c, SD, Z, st);
        case 128: return cols_l<T, 128>(c, SD, Z, st);
        case 256: return cols_l<T, 256>(c, SD, Z, st);
        case 512: return cols_l<T, 512>(c, SD, Z, st);
        case 1024: return cols_l<T, 1024>(c, SD, Z, st);
        case 2048: return cols_l<T, 2048>(c, SD, Z, st);
        case 4096: return cols_l<T, 4096>(c, SD, Z, st);
    }
    set_error("Cartesian column transform of %d points not built", c.Lx);
    return PF_EUNSUPPORTED;
}

template <int L>
int fold_l(const CartPlan &c, const cx<double> *rowspec, cx2<double> *spec, cx<double> *rsp,
           const cx<double> *twL, hipStream_t st) {
    constexpr int E = L >= 4096 ? 16 : 8;
    const size_t lds = (size_t)padded_len(L) * sizeof(cx<double>);
    int rc = allow_lds_cart(k_cart_fold<L, E>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_cart_fold<L, E>), dim3(c.H + 1), dim3(L / E), lds, st, rowspec, c.H,
                       0.5 / c.dx, 1.0 / ((double)c.Lx * (double)c.Ly), spec, rsp, c.ldspec,
                       twL);
    PF_HIP(hipGetLastError());
    return PF_OK;
}

int launch_cart_fold(const CartPlan &c, const cx<double> *rowspec, cx2<double> *spec,
                     cx<double> *rsp, const cx<double> *twL, hipStream_t st) {
    switch (c.Lx) {
        case 8: return fold_l<8>(c, rowspec, spec, rsp, twL, st);
        case 16: return fold_l<16>(c, rowspec, spec, rsp, twL, st);
        case 32: return fold_l<32>(c, rowspec, spec, rsp, twL, st);
        case 64: return fold_l<64>(c, rowspec, spec, rsp, twL, st);
        case 128: return fold_l<128>(c, rowspec, spec, rsp, twL, st);
        case 256: return fold_l<256>(c, rowspec, spec, rsp, twL, st);
        case 512: return fold_l<512>(c, rowspec, spec, rsp, twL, st);
        case 1024: return fold_l<1024>(c, rowspec, spec, rsp, twL, st);
        case 2048: return fold_l<2048>(c, rowspec, spec, rsp, twL, st);
        case 4096: return fold_l<4096>(c, rowspec, spec, rsp, twL, st);
    }
    set_error("Cartesian fold of %d points not built", c.Lx);
    return PF_EUNSUPPORTED;
}

int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int cart_build(CartPlan &c, int dtype, int method, hipStream_t st) {
    free_cart(c);
    c.dtype = dtype;
    c.method = method;
    const bool f64 = dtype == PF_F64;
    const size_t ns = (size_t)2 * c.H * c.ldspec;   // entries per spectrum set
    DevBuf gl, tab, rowspec, spec64, rsp64, twN64, twL64;

    std::vector<double> gx, gw;
    gauss_legendre_host(16, gx, gw);
    std::vector<double> glh(32);
    for (int k = 0; k < 16; ++k) {
        glh[k] = gx[k];
        glh[16 + k] = gw[k];
    }
    PF_HIP(hipMalloc(&gl.p, 32 * sizeof(double)));
    PF_HIP(hipMemcpyAsync(gl.p, glh.data(), 32 * sizeof(double), hipMemcpyHostToDevice, st));

    const size_t plane = (size_t)c.Lx * c.Ly;
    if (hipMalloc(&tab.p, 6 * plane * sizeof(double)) != hipSuccess ||
        hipMalloc(&rowspec.p, 6 * (size_t)c.Lx * c.H * sizeof(cx<double>)) != hipSuccess ||
        hipMalloc(&spec64.p, ns * sizeof(cx2<double>) + kSpecTailPad) != hipSuccess ||
        hipMalloc(&rsp64.p, ns * sizeof(cx<double>)) != hipSuccess) {
        set_error("Cartesian table allocation failed");
        return PF_ENOMEM;
    }
    PF_HIP(hipMemsetAsync(spec64.p, 0, ns * sizeof(cx2<double>), st));
    PF_HIP(hipMemsetAsync(rsp64.p, 0, ns * sizeof(cx<double>), st));
    CartGeo g{c.n_x, c.n_y, c.Lx, c.Ly, method, c.dx, c.dy};
    hipLaunchKernelGGL(k_cart_tables, dim3((c.Ly + 255) / 256, c.Lx), dim3(256), 0, st, g,
                       (const double *)gl.p, (double *)tab.p);
    PF_HIP(hipGetLastError());

    int rc = upload_twiddles(c.Ly, true, &twN64.p);
    if (!rc) rc = upload_twiddles(c.Lx, true, &twL64.p);
    if (rc) return rc;
    {   // row transforms of the six tables along y (FP64)
        Plan rp;
        rp.M = c.H;
        Shape s;
        s.E = c.H >= 2048 ? 16 : (c.H < 8 ? c.H : 8);
        s.G = 1;
        rc = launch_rows_r2c<double>(rp, (const double *)tab.p, nullptr, 6 * c.Lx,
                                     (cx<double> *)rowspec.p, (const cx<double> *)twN64.p, s, st);
        if (rc) return rc;
    }
    rc = launch_cart_fold(c, (const cx<double> *)rowspec.p, (cx2<double> *)spec64.p,
                          (cx<double> *)rsp64.p, (const cx<double> *)twL64.p, st);
    if (rc) return rc;

    if (f64) {
        c.spec = spec64.p;
        c.rsp = rsp64.p;
        spec64.p = rsp64.p = nullptr;
        c.twN = twN64.p;
        c.twL = twL64.p;
        twN64.p = twL64.p = nullptr;
    } else {
        PF_HIP(hipMalloc(&c.spec, ns * sizeof(cx2<float>) + kSpecTailPad));
        PF_HIP(hipMalloc(&c.rsp, ns * sizeof(cx<float>)));
        hipLaunchKernelGGL(k_cart_to_f32, dim3(1024), dim3(256), 0, st,
                           (const double *)spec64.p, (float *)c.spec, (long)(ns * 4));
        hipLaunchKernelGGL(k_cart_to_f32, dim3(1024), dim3(256), 0, st, (const double *)rsp64.p,
                           (float *)c.rsp, (long)(ns * 2));
        PF_HIP(hipGetLastError());
        rc = upload_twiddles(c.Ly, false, &c.twN);
        if (!rc) rc = upload_twiddles(c.Lx, false, &c.twL);
        if (rc) return rc;
    }
    const size_t wsb = ((size_t)2 * c.n_x * c.H * (f64 ? sizeof(cx2<double>) : sizeof(cx2<float>)) +
                        255) / 256 * 256;
    if (hipMalloc(&c.ws, wsb + kScaleSet * sizeof(unsigned)) != hipSuccess) {
        set_error("Cartesian workspace allocation failed");
        return PF_ENOMEM;
    }
    c.gscale = nullptr;
    if (!f64) {   // the notes start at zero; pass C leaves them so
        c.gscale = (unsigned *)((unsigned char *)c.ws + wsb);
        PF_HIP(hipMemsetAsync(c.gscale, 0, kScaleSet * sizeof(unsigned), st));
    }
    PF_HIP(hipStreamSynchronize(st));
    c.rows = cart_rows_shape(c.H);
    c.cols = cart_cols_shape(c.Lx, f64);
    c.built = true;
    return PF_OK;
}

template <typename T>
int cart_forces_t(const CartPlan &c, const T *sigma, T *fx, T *fy, hipStream_t st) {
    cx2<T> *SD = (cx2<T> *)c.ws;
    cx2<T> *Z = SD + (size_t)c.n_x * c.H;
    int rc = launch_cart_rows<T>(c, false, sigma, SD, nullptr, st);
    if (rc) return rc;
    rc = launch_cart_cols<T>(c, SD, Z, st);
    if (rc) return rc;
    return launch_cart_rows<T>(c, true, Z, fx, fy, st);
}

template <typename T>
int cart_timed_t(const CartPlan &c, const T *sigma, T *fx, T *fy, int reps, hipStream_t st,
                 hipEvent_t *ev) {
    cx2<T> *SD = (cx2<T> *)c.ws;
    cx2<T> *Z = SD + (size_t)c.n_x * c.H;
    int rc = PF_OK;
    PF_HIP(hipEventRecord(ev[0], st));
    for (int k = 0; k < reps && !rc; ++k) rc = launch_cart_rows<T>(c, false, sigma, SD, nullptr, st);
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[1], st));
    for (int k = 0; k < reps && !rc; ++k) rc = launch_cart_cols<T>(c, SD, Z, st);
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[2], st));
    for (int k = 0; k < reps && !rc; ++k) rc = launch_cart_rows<T>(c, true, Z, fx, fy, st);
    if (rc) return rc;
    PF_HIP(hipEventRecord(ev[3], st));
    return PF_OK;
}

int cart_device_present() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        set_error("no GPU device available");
        return PF_ENODEV;
    }
    return PF_OK;
}

}  // namespace
}  // namespace pf

struct pf_cart_s {
    pf::CartPlan c;
};

extern "C" {

pf_cart pf_cart_create(int n_x, int n_y, double dx, double dy) {
    pf::clear_error();
    if (n_x < 4 || n_x > 2048 || n_y < 4 || n_y > 2048) {
        pf::set_error("grid %d x %d outside 4..2048 per side", n_x, n_y);
        return nullptr;
    }
    if (!(dx > 0) || !(dy > 0) || !std::isfinite(dx) || !std::isfinite(dy)) {
        pf::set_error("cell sizes must be positive and finite");
        return nullptr;
    }
    pf_cart h = new (std::nothrow) pf_cart_s;
    if (!h) {
        pf::set_error("out of host memory");
        return nullptr;
    }
    pf::CartPlan &c = h->c;
    c.n_x = n_x;
    c.n_y = n_y;
    c.dx = dx;
    c.dy = dy;
    c.Lx = pf::pow2_at_least(2 * n_x);
    c.Ly = pf::pow2_at_least(2 * n_y);
    c.H = c.Ly / 2;
    c.ldspec = c.Lx / 2 + 1;
    return h;
}

int pf_cart_build(pf_cart h, int dtype, int method, void *stream) {
    pf::clear_error();
    if (!h) {
        pf::set_error("null plan");
        return PF_EINVAL;
    }
    if (dtype != PF_F32 && dtype != PF_F64) {
        pf::set_error("dtype must be PF_F32 or PF_F64");
        return PF_EINVAL;
    }
    if (method != PF_CART_SECOND && method != PF_CART_PARTICLE &&
        method != PF_CART_PARTICLE_PLUS) {
        pf::set_error("method must be PF_CART_SECOND, PF_CART_PARTICLE or PF_CART_PARTICLE_PLUS");
        return PF_EINVAL;
    }
    int rc = pf::cart_device_present();
    if (rc) return rc;
    rc = pf::cart_build(h->c, dtype, method, (hipStream_t)stream);
    if (rc) pf::free_cart(h->c);
    return rc;
}

int pf_cart_forces(pf_cart h, const void *sigma, void *f_x, void *f_y, void *stream) {
    pf::clear_error();
    if (!h || !sigma || !f_x || !f_y) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    if (!h->c.built) {
        pf::set_error("plan not built (call pf_cart_build first)");
        return PF_ESTATE;
    }
    hipStream_t st = (hipStream_t)stream;
    if (h->c.dtype == PF_F64)
        return pf::cart_forces_t<double>(h->c, (const double *)sigma, (double *)f_x,
                                         (double *)f_y, st);
    return pf::cart_forces_t<float>(h->c, (const float *)sigma, (float *)f_x, (float *)f_y, st);
}

int pf_cart_forces_timed(pf_cart h, const void *sigma, void *f_x, void *f_y, int reps,
                         void *stream, float *pass_ms) {
    pf::clear_error();
    if (!h || !sigma || !f_x || !f_y || !pass_ms) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    if (reps < 1 || reps > 10000) {
        pf::set_error("reps must be in 1..10000");
        return PF_EINVAL;
    }
    if (!h->c.built) {
        pf::set_error("plan not built (call pf_cart_build first)");
        return PF_ESTATE;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int rc = PF_OK;
    for (int k = 0; k < 4 && !rc; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) {
            pf::set_error("hipEventCreate failed");
            rc = PF_EHIP;
        }
    if (!rc)
        rc = h->c.dtype == PF_F64
                 ? pf::cart_timed_t<double>(h->c, (const double *)sigma, (double *)f_x,
                                            (double *)f_y, reps, st, ev)
                 : pf::cart_timed_t<float>(h->c, (const float *)sigma, (float *)f_x,
                                           (float *)f_y, reps, st, ev);
    if (!rc && hipEventSynchronize(ev[3]) != hipSuccess) {
        pf::set_error("hipEventSynchronize failed");
        rc = PF_EHIP;
    }
    for (int k = 0; k < 3 && !rc; ++k) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) {
            pf::set_error("hipEventElapsedTime failed");
            rc = PF_EHIP;
        }
        pass_ms[k] = ms / reps;
    }
    for (int k = 0; k < 4; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
    return rc;
}

int pf_cart_geometry(pf_cart h, int out[4]) {
    pf::clear_error();
    if (!h || !out) {
        pf::set_error("null argument");
        return PF_EINVAL;
    }
    out[0] = h->c.n_x;
    out[1] = h->c.n_y;
    out[2] = h->c.Lx;
    out[3] = h->c.Ly;
    return PF_OK;
}

void pf_cart_destroy(pf_cart h) {
    if (!h) return;
    pf::free_cart(h->c);
    delete h;
}

}  // extern "C"
