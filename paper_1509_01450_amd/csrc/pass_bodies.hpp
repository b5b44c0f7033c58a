// pass_bodies.hpp -- device bodies of the per-call passes, shared by the
// standalone kernels (pf_passes.hip) and the persistent batched kernel
// (pf_batched.hip).  Each body processes one "unit" (a group of G rows or G
// columns) with the calling workgroup; every thread of the workgroup must
// call it (the bodies contain barriers).
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
#pragma once
#include "fft_core.hpp"

namespace pf {

// ---------------------------------------------------------------------------
// Pass A: real-to-complex transforms of rows of length N = 2M via one
// M-point complex transform of z[n] = x[2n] + i x[2n+1].
// Workgroup: G rows x (M/E) threads; LDS buf: G*padded_len(M) complex.
// ---------------------------------------------------------------------------
template <typename T, int M, int E>
__device__ __forceinline__ void body_rows_r2c(int unit, int G, cx<T> *__restrict__ buf,
                                           const T *__restrict__ in0,
                                                  const T *__restrict__ in1, int n_rows,
                                                  int total_rows, cx<T> *__restrict__ out0,
                                                  cx<T> *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    constexpr int H = M + 1;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < total_rows;
    const int arr = active ? row / n_rows : 0;
    const int i = active ? row % n_rows : 0;   // inactive lanes read row 0
    const T *x = (arr == 0 ? in0 : in1) + (size_t)i * N;
    cx<T> *out = (arr == 0 ? out0 : out1) + (size_t)i * H;
    Lds<T> lds{buf, gi * padded_len(M), 1};

    // unconditional loads (in bounds for every lane) so they issue together
    cx<T> v[E];
    const cx<T> *xz = reinterpret_cast<const cx<T> *>(x);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xz[t + e * TH];
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (!active) v[e] = cx<T>{T(0), T(0)};
    fft_fwd<M, E, T>(v, t, lds, tw);
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
__device__ __forceinline__ void body_rows_c2r(int unit, int G, cx<T> *__restrict__ buf,
                                           const cx<T> *__restrict__ in0,
                                                  const cx<T> *__restrict__ in1, int n_rows,
                                                  int total_rows, T *__restrict__ out0,
                                                  T *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    constexpr int H = M + 1;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < total_rows;
    const int arr = active ? row / n_rows : 0;
    const int i = active ? row % n_rows : 0;   // inactive lanes read row 0
    const cx<T> *X = (arr == 0 ? in0 : in1) + (size_t)i * H;
    T *y = (arr == 0 ? out0 : out1) + (size_t)i * N;
    Lds<T> lds{buf, gi * padded_len(M), 1};

    // unconditional loads (in bounds for every lane) so they issue together
    cx<T> xk[E], xm[E], wk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
        xk[e] = X[k];
        xm[e] = X[M - k];
        wk[e] = twN[k];                          // exp(-2 pi i k / N)
    }
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        cx<T> s = {xk[e].x + xm[e].x, xk[e].y - xm[e].y};   // X[k] + conj X[M-k]
        cx<T> d = {xk[e].x - xm[e].x, xk[e].y + xm[e].y};   // X[k] - conj X[M-k]
        cx<T> dw = cmulc(d, wk[e]);                           // d * exp(+2 pi i k / N)
        v[e] = active ? cx<T>{s.x - dw.y, s.y + dw.x} : cx<T>{T(0), T(0)};   // s + i dw
    }
    fft_inv<M, E, T>(v, t, lds, tw);
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
    const bool lo = ku <= HL;
    const cx<T> s = col[lo ? ku : L - ku];   // one load, no branch
    if (lo) return s;
    return odd ? cx<T>{-s.x, s.y} : cx<T>{s.x, -s.y};
}

// ---------------------------------------------------------------------------
// Pass B, forward.  Workgroup: G columns x (L/E) threads, lane -> (t, column)
// with the G columns interleaved (consecutive lanes read consecutive
// columns of a row).  LDS buf: G*padded_len(L) complex.
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
__device__ __forceinline__ void body_cols_fwd(int unit, int G, cx<T> *__restrict__ buf,
                                           const cx<T> *__restrict__ S,
                                                  cx<T> *__restrict__ Zr, cx<T> *__restrict__ Zp,
                                                  const cx<T> *__restrict__ spec, int H, int n_r,
                                                  int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL) {
    constexpr int TH = L / E;
    const int grp = unit;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = grp * G + gi;
    const bool valid = col < H;
    Lds<T> lds{buf, gi, G};

    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
    // stage the column in LDS to form the radial slope channel.  Only the
    // first E/2 points of a thread can be data rows (L >= 2 n_r); the loads
    // use clamped, always valid addresses so they issue back to back.
    {
        const int cl = valid ? col : 0;
        cx<T> g[E / 2];
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int i = t + e * TH;
            g[e] = S[(size_t)(i < n_r ? i : n_r - 1) * H + cl];
        }
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int i = t + e * TH;
            if (i < n_r) lds.st(i, valid ? g[e] : cx<T>{T(0), T(0)});
        }
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
    fft_fwd<L, E, T>(vc, t, lds, tw);
    fft_fwd<L, E, T>(vg, t, lds, tw);
    const int cs = valid ? col : 0;
    const cx<T> *er = spec + (size_t)(0 * H + cs) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cs) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cs) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cs) * ldspec;
    // all spectrum loads of the unit in one batch (one memory round trip)
    cx<T> sa[E], sb[E], sc[E], sd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int ku = t + e * TH;
        sa[e] = spec_at<T, L>(er, ku, false);
        sb[e] = spec_at<T, L>(qr, ku, false);
        sc[e] = spec_at<T, L>(ep, ku, true);
        sd[e] = spec_at<T, L>(qp, ku, true);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        cx<T> x = vc[e], y = vg[e];
        vc[e] = cmul(sa[e], x) + cmul(sb[e], y);
        vg[e] = cmul(sc[e], x) + cmul(sd[e], y);
    }
    fft_inv<L, E, T>(vc, t, lds, tw);
    fft_inv<L, E, T>(vg, t, lds, tw);
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
__device__ __forceinline__ void body_cols_adj(int unit, int G, cx<T> *__restrict__ buf,
                                           const cx<T> *__restrict__ Vr,
                                                  const cx<T> *__restrict__ Vp,
                                                  cx<T> *__restrict__ D,
                                                  const cx<T> *__restrict__ spec, int H, int n_r,
                                                  int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL) {
    constexpr int TH = L / E;
    const int grp = unit;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = grp * G + gi;
    const bool valid = col < H;
    Lds<T> lds{buf, gi, G};

    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
    // clamped, always valid addresses so the loads issue back to back; only
    // the first E/2 points of a thread can be data rows (L >= 2 n_r)
    cx<T> va[E], vb[E];
    {
        const int cl = valid ? col : 0;
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int i = t + e * TH;
            const size_t o = (size_t)(i < n_r ? i : n_r - 1) * H + cl;
            va[e] = Vr[o];
            vb[e] = Vp[o];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + e * TH;
            const bool in = valid && i < n_r && e < E / 2;
            if (!in) {
                va[e] = cx<T>{T(0), T(0)};
                vb[e] = cx<T>{T(0), T(0)};
            }
        }
    }
    fft_fwd<L, E, T>(va, t, lds, tw);
    fft_fwd<L, E, T>(vb, t, lds, tw);
    const int cs = valid ? col : 0;
    const cx<T> *er = spec + (size_t)(0 * H + cs) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cs) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cs) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cs) * ldspec;
    // all spectrum loads of the unit in one batch (one memory round trip)
    cx<T> sa[E], sb[E], sc[E], sd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int ku = t + e * TH;
        sa[e] = spec_at<T, L>(er, ku, false);
        sb[e] = spec_at<T, L>(qr, ku, false);
        sc[e] = spec_at<T, L>(ep, ku, true);
        sd[e] = spec_at<T, L>(qp, ku, true);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        cx<T> x = va[e], y = vb[e];
        va[e] = cmulc(x, sa[e]) + cmulc(y, sc[e]);   // conj(E_r) v_r + conj(E_p) v_p
        vb[e] = cmulc(x, sb[e]) + cmulc(y, sd[e]);   // conj(Q_r) v_r + conj(Q_p) v_p
    }
    fft_inv<L, E, T>(va, t, lds, tw);
    fft_inv<L, E, T>(vb, t, lds, tw);
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

}  // namespace pf
