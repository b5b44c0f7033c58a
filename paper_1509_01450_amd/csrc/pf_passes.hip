// pf_passes.hip -- the per-call hot path: row transforms along phi and the
// fused column pass along u = ln r, forward and transpose.
//
// Forward map (Eq. 26-29, A18-A21) as a 2-D convolution:
//   pass A  S = R2C_phi(sigma)                         rows,    [n_r][H]
//   pass B  per column k:  c = S[:, k], g = D_r c (radial slope, Eq. 25)
//           Zr = crop IFFT_u(E_r FFT_u(pad c) + Q_r FFT_u(pad g))
//           Zp = crop IFFT_u(E_p FFT_u(pad c) + Q_p FFT_u(pad g))
//   pass C  F_r = C2R_phi(Zr), F_phi = C2R_phi(Zp)
// The azimuthal slope channel is folded into E_r, E_p (exact for the
// periodic central difference), the r_i / r_i' = beta^(i-i') factor of
// Eq. 28 into Q_r, Q_p; g = r delta^r.  Padding to L >= 2 n_r in u makes the
// circular convolution equal the linear one on the n_r output rows, so no
// artificial boundary condition enters (Sec. 2).
//
// Layouts: S, Zr, Zp, Vr, Vp, D are row-major [n_r][H] complex, H = n_phi/2+1;
// spectra are [4][H][L/2+1] complex (E_r, Q_r, E_p, Q_p), column-contiguous,
// holding k_u in [0, L/2]; the rest follows from the kernels' symmetry in phi.
#include "pf_common.hpp"

namespace pf {

// ---------------------------------------------------------------------------
// Pass A: real-to-complex transforms of rows of length N = 2M via one
// M-point complex transform of z[n] = x[2n] + i x[2n+1].
// Block: G rows x (M/E) threads; dynamic LDS G*M complex.
// ---------------------------------------------------------------------------
template <typename T, int M, int E>
__global__ __launch_bounds__(512) void k_rows_r2c(const T *__restrict__ in0,
                                                  const T *__restrict__ in1, int n_rows,
                                                  int total_rows, cx<T> *__restrict__ out0,
                                                  cx<T> *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    constexpr int H = M + 1;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int G = blockDim.x / TH;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = blockIdx.x * G + gi;
    const bool active = row < total_rows;
    const int arr = active ? row / n_rows : 0;
    const int i = active ? row % n_rows : 0;
    const T *x = (arr == 0 ? in0 : in1) + (size_t)i * N;
    cx<T> *out = (arr == 0 ? out0 : out1) + (size_t)i * H;
    Lds<T> lds{buf, gi * M, 1};

    cx<T> v[E];
    const cx<T> *xz = reinterpret_cast<const cx<T> *>(x);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? xz[t + e * TH] : cx<T>{T(0), T(0)};
    fft_fwd<M, E, T>(v, t, lds, twN, 2);
#pragma unroll
    for (int e = 0; e < E; ++e) lds.st(t + e * TH, v[e]);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            cx<T> zk = lds.ld(k), zm = lds.ld((M - k) & (M - 1));
            cx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            // (zk - conj zm) / (2i)
            cx<T> od = {T(0.5) * (zk.y + zm.y), -T(0.5) * (zk.x - zm.x)};
            out[k] = ev + cmul(twN[k], od);
        }
        if (t == 0) {
            cx<T> z0 = lds.ld(0);
            out[M] = cx<T>{z0.x - z0.y, T(0)};
        }
    }
}

// ---------------------------------------------------------------------------
// Pass C: complex-to-real transforms of Hermitian half rows (H values) to
// real rows of length N = 2M (unnormalised inverse).
// ---------------------------------------------------------------------------
template <typename T, int M, int E>
__global__ __launch_bounds__(512) void k_rows_c2r(const cx<T> *__restrict__ in0,
                                                  const cx<T> *__restrict__ in1, int n_rows,
                                                  int total_rows, T *__restrict__ out0,
                                                  T *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    constexpr int H = M + 1;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int G = blockDim.x / TH;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = blockIdx.x * G + gi;
    const bool active = row < total_rows;
    const int arr = active ? row / n_rows : 0;
    const int i = active ? row % n_rows : 0;
    const cx<T> *X = (arr == 0 ? in0 : in1) + (size_t)i * H;
    T *y = (arr == 0 ? out0 : out1) + (size_t)i * N;
    Lds<T> lds{buf, gi * M, 1};

    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
        if (active) {
            cx<T> xk = X[k], xm = X[M - k];
            cx<T> s = {xk.x + xm.x, xk.y - xm.y};   // X[k] + conj X[M-k]
            cx<T> d = {xk.x - xm.x, xk.y + xm.y};   // X[k] - conj X[M-k]
            cx<T> w = twN[k];                        // exp(-2 pi i k / N)
            cx<T> dw = cmulc(d, w);                  // d * exp(+2 pi i k / N)
            v[e] = cx<T>{s.x - dw.y, s.y + dw.x};    // s + i dw
        } else {
            v[e] = cx<T>{T(0), T(0)};
        }
    }
    fft_inv<M, E, T>(v, t, lds, twN, 2);
    if (active) {
        cx<T> *yz = reinterpret_cast<cx<T> *>(y);
#pragma unroll
        for (int e = 0; e < E; ++e) yz[t + e * TH] = v[e];
    }
}

// ---------------------------------------------------------------------------
// Spectrum access with the phi-parity symmetry of the kernels:
// E_r, Q_r even in n -> value at -k_u is conj; E_p, Q_p odd -> -conj.
// ---------------------------------------------------------------------------
template <typename T, int L>
__device__ __forceinline__ cx<T> spec_at(const cx<T> *__restrict__ col, int ku, bool odd) {
    constexpr int HL = L / 2;
    if (ku <= HL) return col[ku];
    cx<T> s = col[L - ku];
    return odd ? cx<T>{-s.x, s.y} : cx<T>{s.x, -s.y};
}

// Column-group index with the groups of one XCD contiguous: workgroups are
// dispatched round-robin over the 8 XCDs, so block b runs on XCD b % 8.
__device__ __forceinline__ int xcd_group(int b, int per_xcd) { return (b & 7) * per_xcd + (b >> 3); }

// ---------------------------------------------------------------------------
// Pass B, forward.  Block: G columns x (L/E) threads, lane -> (t, column)
// with the G columns interleaved (consecutive lanes read consecutive
// columns of a row).  Dynamic LDS: L*G complex.
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
__global__ __launch_bounds__(512) void k_cols_fwd(const cx<T> *__restrict__ S,
                                                  cx<T> *__restrict__ Zr, cx<T> *__restrict__ Zp,
                                                  const cx<T> *__restrict__ spec, int H, int n_r,
                                                  int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL, int per_xcd,
                                                  int n_groups) {
    constexpr int TH = L / E;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int G = blockDim.x / TH;
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;  // whole block leaves together
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = grp * G + gi;
    const bool valid = col < H;
    Lds<T> lds{buf, gi, G};

    // stage the column in LDS to form the radial slope channel
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (i < n_r) lds.st(i, valid ? S[(size_t)i * H + col] : cx<T>{T(0), T(0)});
    }
    __syncthreads();
    cx<T> vc[E], vg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        cx<T> c = {T(0), T(0)}, g = {T(0), T(0)};
        if (i < n_r) {
            c = lds.ld(i);
            if (i == 0)
                g = scale(lds.ld(1) - c, c0);
            else if (i == n_r - 1)
                g = scale(c - lds.ld(i - 1), cn);
            else
                g = scale(lds.ld(i + 1) - lds.ld(i - 1), ca);
        }
        vc[e] = c;
        vg[e] = g;
    }
    __syncthreads();
    fft_fwd<L, E, T>(vc, t, lds, twL, 1);
    fft_fwd<L, E, T>(vg, t, lds, twL, 1);
    const int cs = valid ? col : 0;
    const cx<T> *er = spec + (size_t)(0 * H + cs) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cs) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cs) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cs) * ldspec;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int ku = t + e * TH;
        cx<T> a = spec_at<T, L>(er, ku, false), b = spec_at<T, L>(qr, ku, false);
        cx<T> c = spec_at<T, L>(ep, ku, true), d = spec_at<T, L>(qp, ku, true);
        cx<T> x = vc[e], y = vg[e];
        vc[e] = cmul(a, x) + cmul(b, y);
        vg[e] = cmul(c, x) + cmul(d, y);
    }
    fft_inv<L, E, T>(vc, t, lds, twL, 1);
    fft_inv<L, E, T>(vg, t, lds, twL, 1);
    if (valid) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + e * TH;
            if (i < n_r) {
                Zr[(size_t)i * H + col] = vc[e];
                Zp[(size_t)i * H + col] = vg[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass B, transpose: correlate with the kernels (conjugate spectra), then
// apply the transposed radial-slope stencil: d = c_s + D_r^T c_g.
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
__global__ __launch_bounds__(512) void k_cols_adj(const cx<T> *__restrict__ Vr,
                                                  const cx<T> *__restrict__ Vp,
                                                  cx<T> *__restrict__ D,
                                                  const cx<T> *__restrict__ spec, int H, int n_r,
                                                  int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL, int per_xcd,
                                                  int n_groups) {
    constexpr int TH = L / E;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int G = blockDim.x / TH;
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = grp * G + gi;
    const bool valid = col < H;
    Lds<T> lds{buf, gi, G};

    cx<T> va[E], vb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        const bool in = valid && i < n_r;
        va[e] = in ? Vr[(size_t)i * H + col] : cx<T>{T(0), T(0)};
        vb[e] = in ? Vp[(size_t)i * H + col] : cx<T>{T(0), T(0)};
    }
    fft_fwd<L, E, T>(va, t, lds, twL, 1);
    fft_fwd<L, E, T>(vb, t, lds, twL, 1);
    const int cs = valid ? col : 0;
    const cx<T> *er = spec + (size_t)(0 * H + cs) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cs) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cs) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cs) * ldspec;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int ku = t + e * TH;
        cx<T> a = spec_at<T, L>(er, ku, false), b = spec_at<T, L>(qr, ku, false);
        cx<T> c = spec_at<T, L>(ep, ku, true), d = spec_at<T, L>(qp, ku, true);
        cx<T> x = va[e], y = vb[e];
        va[e] = cmulc(x, a) + cmulc(y, c);   // conj(E_r) v_r + conj(E_p) v_p
        vb[e] = cmulc(x, b) + cmulc(y, d);   // conj(Q_r) v_r + conj(Q_p) v_p
    }
    fft_inv<L, E, T>(va, t, lds, twL, 1);
    fft_inv<L, E, T>(vb, t, lds, twL, 1);
    // transposed stencil on the slope channel
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (i < n_r) lds.st(i, vb[e]);
    }
    __syncthreads();
    if (valid) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + e * TH;
            if (i < n_r) {
                cx<T> acc = va[e];
                if (i >= 1) acc = acc + scale(lds.ld(i - 1), i == 1 ? c0 : ca);
                if (i <= n_r - 2) acc = acc - scale(lds.ld(i + 1), i == n_r - 2 ? cn : ca);
                if (i == 0) acc = acc - scale(lds.ld(0), c0);
                if (i == n_r - 1) acc = acc + scale(lds.ld(n_r - 1), cn);
                D[(size_t)i * H + col] = acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Runtime dispatch onto the template instantiations.
// ---------------------------------------------------------------------------
bool valid_shape_rows(int M, Shape s, bool f64) {
    if (!(s.E == 4 || s.E == 8 || s.E == 16) || s.E > M) return false;
    const int th = M / s.E;
    if (s.G < 1 || th * s.G > 512) return false;
    const size_t lds = (size_t)s.G * M * (f64 ? 16 : 8);
    return lds <= 64 * 1024;
}

bool valid_shape_cols(int L, Shape s, bool f64) {
    if (!(s.E == 8 || s.E == 16) || s.E > L) return false;
    const int th = L / s.E;
    if (s.G < 1 || th * s.G > 512) return false;
    const size_t lds = (size_t)s.G * L * (f64 ? 16 : 8);
    return lds <= 128 * 1024;
}

#define PF_SWITCH_POW2(v, F, ...)                          \
    switch (v) {                                           \
        case 4: return F<4>(__VA_ARGS__);                  \
        case 8: return F<8>(__VA_ARGS__);                  \
        case 16: return F<16>(__VA_ARGS__);                \
        case 32: return F<32>(__VA_ARGS__);                \
        case 64: return F<64>(__VA_ARGS__);                \
        case 128: return F<128>(__VA_ARGS__);              \
        case 256: return F<256>(__VA_ARGS__);              \
        case 512: return F<512>(__VA_ARGS__);              \
        case 1024: return F<1024>(__VA_ARGS__);            \
        case 2048: return F<2048>(__VA_ARGS__);            \
        case 4096: return F<4096>(__VA_ARGS__);            \
        case 8192: return F<8192>(__VA_ARGS__);            \
        default: set_error("unsupported transform length %d", v); return PF_EUNSUPPORTED; \
    }

namespace {

template <typename K>
int allow_lds(K kern, size_t lds) {
    if (lds > 64 * 1024)
        PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PF_OK;
}

template <typename T>
struct Disp {
    template <int N, int E>
    static int r2c(const T *in0, const T *in1, int n_arr, int n_rows, cx<T> *o0, cx<T> *o1,
                   const cx<T> *tw, int G, hipStream_t st) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int total = n_arr * n_rows;
            const int blocks = (total + G - 1) / G;
            const size_t lds = (size_t)G * N * sizeof(cx<T>);
            hipLaunchKernelGGL((k_rows_r2c<T, N, E>), dim3(blocks), dim3(G * TH), lds, st, in0,
                               in1, n_rows, total, o0, o1, tw);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N, int E>
    static int c2r(const cx<T> *in0, const cx<T> *in1, int n_arr, int n_rows, T *o0, T *o1,
                   const cx<T> *tw, int G, hipStream_t st) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int total = n_arr * n_rows;
            const int blocks = (total + G - 1) / G;
            const size_t lds = (size_t)G * N * sizeof(cx<T>);
            hipLaunchKernelGGL((k_rows_c2r<T, N, E>), dim3(blocks), dim3(G * TH), lds, st, in0,
                               in1, n_rows, total, o0, o1, tw);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N, int E, bool ADJ>
    static int cols(const Plan &p, const cx<T> *a, const cx<T> *b, cx<T> *o0, cx<T> *o1,
                    const cx<T> *spec, const cx<T> *tw, int G, hipStream_t st) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int n_groups = (p.H + G - 1) / G;
            const int per_xcd = (n_groups + 7) / 8;
            const int blocks = per_xcd * 8;
            const size_t lds = (size_t)G * N * sizeof(cx<T>);
            const T ca = T(p.ca), c0 = T(p.c0), cn = T(p.cn);
            if (ADJ) {
                int rc = allow_lds(k_cols_adj<T, N, E>, lds);
                if (rc) return rc;
                hipLaunchKernelGGL((k_cols_adj<T, N, E>), dim3(blocks), dim3(G * TH), lds, st,
                                   a, b, o0, spec, p.H, p.n_r, p.ldspec, ca, c0, cn, tw,
                                   per_xcd, n_groups);
            } else {
                int rc = allow_lds(k_cols_fwd<T, N, E>, lds);
                if (rc) return rc;
                hipLaunchKernelGGL((k_cols_fwd<T, N, E>), dim3(blocks), dim3(G * TH), lds, st,
                                   a, o0, o1, spec, p.H, p.n_r, p.ldspec, ca, c0, cn, tw,
                                   per_xcd, n_groups);
            }
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("column transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int r2c_e(int E, const T *in0, const T *in1, int n_arr, int n_rows, cx<T> *o0,
                     cx<T> *o1, const cx<T> *tw, int G, hipStream_t st) {
        switch (E) {
            case 4: return r2c<N, 4>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
            case 8: return r2c<N, 8>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
            case 16: return r2c<N, 16>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int c2r_e(int E, const cx<T> *in0, const cx<T> *in1, int n_arr, int n_rows, T *o0,
                     T *o1, const cx<T> *tw, int G, hipStream_t st) {
        switch (E) {
            case 4: return c2r<N, 4>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
            case 8: return c2r<N, 8>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
            case 16: return c2r<N, 16>(in0, in1, n_arr, n_rows, o0, o1, tw, G, st);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int fwd_e(int E, const Plan &p, const cx<T> *a, cx<T> *o0, cx<T> *o1,
                     const cx<T> *spec, const cx<T> *tw, int G, hipStream_t st) {
        switch (E) {
            case 8: return cols<N, 8, false>(p, a, nullptr, o0, o1, spec, tw, G, st);
            case 16: return cols<N, 16, false>(p, a, nullptr, o0, o1, spec, tw, G, st);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int adj_e(int E, const Plan &p, const cx<T> *a, const cx<T> *b, cx<T> *o0,
                     const cx<T> *spec, const cx<T> *tw, int G, hipStream_t st) {
        switch (E) {
            case 8: return cols<N, 8, true>(p, a, b, o0, nullptr, spec, tw, G, st);
            case 16: return cols<N, 16, true>(p, a, b, o0, nullptr, spec, tw, G, st);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
};

}  // namespace

template <typename T>
int launch_rows_r2c(const Plan &p, const T *in0, const T *in1, int n_arr, int n_rows,
                    cx<T> *out0, cx<T> *out1, const cx<T> *twN, Shape s, hipStream_t st) {
    if (!valid_shape_rows(p.M, s, sizeof(T) == 8)) {
        set_error("invalid row shape E=%d G=%d for M=%d", s.E, s.G, p.M);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.M, Disp<T>::template r2c_e, s.E, in0, in1, n_arr, n_rows, out0, out1, twN,
                   s.G, st);
}

template <typename T>
int launch_rows_c2r(const Plan &p, const cx<T> *in0, const cx<T> *in1, int n_arr, int n_rows,
                    T *out0, T *out1, const cx<T> *twN, Shape s, hipStream_t st) {
    if (!valid_shape_rows(p.M, s, sizeof(T) == 8)) {
        set_error("invalid row shape E=%d G=%d for M=%d", s.E, s.G, p.M);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.M, Disp<T>::template c2r_e, s.E, in0, in1, n_arr, n_rows, out0, out1, twN,
                   s.G, st);
}

template <typename T>
int launch_cols_fwd(const Plan &p, const cx<T> *S, cx<T> *Zr, cx<T> *Zp, const cx<T> *spec,
                    const cx<T> *twL, Shape s, hipStream_t st) {
    if (!valid_shape_cols(p.L, s, sizeof(T) == 8)) {
        set_error("invalid column shape E=%d G=%d for L=%d", s.E, s.G, p.L);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.L, Disp<T>::template fwd_e, s.E, p, S, Zr, Zp, spec, twL, s.G, st);
}

template <typename T>
int launch_cols_adj(const Plan &p, const cx<T> *Vr, const cx<T> *Vp, cx<T> *D,
                    const cx<T> *spec, const cx<T> *twL, Shape s, hipStream_t st) {
    if (!valid_shape_cols(p.L, s, sizeof(T) == 8)) {
        set_error("invalid column shape E=%d G=%d for L=%d", s.E, s.G, p.L);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.L, Disp<T>::template adj_e, s.E, p, Vr, Vp, D, spec, twL, s.G, st);
}

template int launch_rows_r2c<float>(const Plan &, const float *, const float *, int, int,
                                    cx<float> *, cx<float> *, const cx<float> *, Shape, hipStream_t);
template int launch_rows_r2c<double>(const Plan &, const double *, const double *, int, int,
                                     cx<double> *, cx<double> *, const cx<double> *, Shape,
                                     hipStream_t);
template int launch_rows_c2r<float>(const Plan &, const cx<float> *, const cx<float> *, int, int,
                                    float *, float *, const cx<float> *, Shape, hipStream_t);
template int launch_rows_c2r<double>(const Plan &, const cx<double> *, const cx<double> *, int,
                                     int, double *, double *, const cx<double> *, Shape,
                                     hipStream_t);
template int launch_cols_fwd<float>(const Plan &, const cx<float> *, cx<float> *, cx<float> *,
                                    const cx<float> *, const cx<float> *, Shape, hipStream_t);
template int launch_cols_fwd<double>(const Plan &, const cx<double> *, cx<double> *,
                                     cx<double> *, const cx<double> *, const cx<double> *, Shape,
                                     hipStream_t);
template int launch_cols_adj<float>(const Plan &, const cx<float> *, const cx<float> *,
                                    cx<float> *, const cx<float> *, const cx<float> *, Shape,
                                    hipStream_t);
template int launch_cols_adj<double>(const Plan &, const cx<double> *, const cx<double> *,
                                     cx<double> *, const cx<double> *, const cx<double> *, Shape,
                                     hipStream_t);

}  // namespace pf
