// pass_bodies.hpp -- device bodies of the per-call passes, shared by the
// standalone kernels (pf_passes.hip) and the persistent batched kernel
// (pf_batched.hip).  Each body processes one "unit" (a group of G rows or G
// columns) with the calling workgroup; every thread of the workgroup must
// call it (the bodies contain barriers).
//
// Forward map (Eq. 26-29, A18-A21) as a 2-D convolution:
//   pass A  S = R2C_phi(sigma)                         rows,    [n_r][M]
//   pass B  per column k:  c = S[:, k]
//           Zr = crop IFFT_u(E'_r FFT_u(pad c) + Q_r B(c))
//           Zp = crop IFFT_u(E'_p FFT_u(pad c) + Q_p B(c))
//   pass C  F_r = C2R_phi(Zr), F_phi = C2R_phi(Zp)
// The azimuthal slope channel is folded into E_r, E_p (exact for the
// periodic central difference), the r_i / r_i' = beta^(i-i') factor of
// Eq. 28 into Q_r, Q_p.  The radial slope g = r delta^r c (Eq. 25, constant
// coefficients on the logarithmic grid) is applied in the spectral domain:
// on the zero-padded column it equals the circular central difference
// ca (c[i+1] - c[i-1]) except at four rows (0, n-1, n, L-1), so
//   FFT_u(pad g)[k] = 2i ca sin(2 pi k / L) FFT_u(pad c)[k] + B(c)[k]
// with B(c) the transform of that four-row correction.  The first term is
// folded into the spectra, E' = E + Q * 2i ca sin(2 pi k / L); B(c) costs a
// few complex products per point instead of a second column transform.
// Padding to L >= 2 n_r in u makes the circular convolution equal the
// linear one on the n_r output rows, so no artificial boundary condition
// enters (Sec. 2).
//
// Packed half spectrum: a real row of N = 2M points has M + 1 independent
// bins of which bin 0 and bin M are real; they travel together as the one
// complex value (X_0, X_M) in column 0, so every row holds exactly M complex
// values.  Along u the column 0 data are then c_0 + i c_M with c_0, c_M real
// sequences; pass B separates their transforms with the conjugate mirror
// k -> L - k.  The azimuthal spectra vanish at bins 0 and M (the kernels
// K^{phi,*} are odd in phi - phi'), so column 0 carries the radial spectra
// of both bins and its F_phi output is zero.
//
// Layouts: S, Zr, Zp, Vr, Vp, D are row-major [n_r][M] complex, M = n_phi/2;
// spectra are [4][M][L/2+1] complex (slots E'_r, Q_r, E'_p, Q_p; for
// column 0: E'_r, Q_r of bin 0, E'_r, Q_r of bin M), column-contiguous,
// holding k_u in [0, L/2]; the rest follows from the kernels' symmetry in
// phi.
#pragma once
#include "fft_core.hpp"

namespace pf {

// ---------------------------------------------------------------------------
// Pass A: real-to-complex transforms of rows of length N = 2M via one
// M-point complex transform of z[n] = x[2n] + i x[2n+1]; output in the
// packed half spectrum (bin 0 = (X_0, X_M)).
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
    constexpr int H = M;
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
            cx<T> o = ev + cmul(twN[k], od);
            if (k == 0) o = cx<T>{zk.x + zk.y, zk.x - zk.y};   // (X_0, X_M), both real
            out[k] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// Pass C: complex-to-real transforms of packed half rows (M values, bin 0 =
// (X_0, X_M)) to real rows of length N = 2M (unnormalised inverse).
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
    constexpr int H = M;
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
        xm[e] = X[(M - k) & (M - 1)];
        wk[e] = twN[k];                          // exp(-2 pi i k / N)
    }
    if (t == 0) {   // unpack bin 0 = (X_0, X_M)
        const cx<T> p = xk[0];
        xk[0] = cx<T>{p.x, T(0)};
        xm[0] = cx<T>{p.y, T(0)};
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
// Four-row correction of the radial slope (see the header).  For the column
// c (n = n_r rows, zero beyond) the slope differs from the circular central
// difference at
//   row 0      a0  = c0 (c1 - c0) - ca c1
//   row n - 1  an1 = cn (c[n-1] - c[n-2]) + ca c[n-2]
//   row n      an  = ca c[n-1]
//   row L - 1  am1 = -ca c0
// (c0, ca, cn: the first, interior and last row coefficients).  Its
// transform at k, W = exp(-2 pi i / L), is
//   a0 + am1 W^-k + an W^(n k) + an1 W^((n-1) k).
// A thread holds k = t + e TH, e < E, with W^(j k) = W^(j t) W^(j e TH) and
// W^(j e TH) = r((j e) mod E), r(q) = exp(-2 pi i q / E) an E-th root of
// unity, the same for the whole workgroup.  So per thread
//   b1 = an W^(n t),  b2 = am1 W^-t,  b3 = an1 W^((n-1) t)
// and per point
//   a0 + b1 r(n e) + b2 conj(r(e)) + b3 r((n-1) e).
// ---------------------------------------------------------------------------
template <typename T>
struct SlopeFix {
    cx<T> a0, am1, an, an1;
};

template <typename T>
__device__ __forceinline__ SlopeFix<T> slope_fix(cx<T> x0, cx<T> x1, cx<T> xm2, cx<T> xm1, T ca,
                                                 T c0, T cn) {
    SlopeFix<T> s;
    s.a0 = scale(x1 - x0, c0) - scale(x1, ca);
    s.an1 = scale(xm1 - xm2, cn) + scale(xm2, ca);
    s.an = scale(xm1, ca);
    s.am1 = scale(x0, -ca);
    return s;
}

// real or imaginary parts of the coefficients (one bin of packed column 0)
template <typename T>
__device__ __forceinline__ SlopeFix<T> slope_fix_part(const SlopeFix<T> &s, bool imag) {
    auto pick = [imag](cx<T> a) { return cx<T>{imag ? a.y : a.x, T(0)}; };
    return {pick(s.a0), pick(s.am1), pick(s.an), pick(s.an1)};
}

template <typename T>
struct SlopePhasors {
    cx<T> a0, b1, b2, b3;
};

// wt = W^t, wnt = W^(n t), both from the L-point table
template <typename T>
__device__ __forceinline__ SlopePhasors<T> slope_phasors(const SlopeFix<T> &s, cx<T> wt,
                                                         cx<T> wnt) {
    const cx<T> wtc = conj(wt);
    return {s.a0, cmul(s.an, wnt), cmul(s.am1, wtc), cmul(s.an1, cmul(wnt, wtc))};
}

// E-th roots of unity the workgroup needs for point e: r(e), r(n e),
// r((n-1) e), read from the L-point table (r(q) = W^(q L / E)) at addresses
// that are the same for every lane
template <typename T, int L, int E>
struct Roots {
    cx<T> r1, rn, rm;
    __device__ __forceinline__ Roots(const cx<T> *__restrict__ twL, int n, int e) {
        constexpr int TH = L / E;
        r1 = twL[(e & (E - 1)) * TH];
        rn = twL[((n * e) & (E - 1)) * TH];
        rm = twL[(((n - 1) * e) & (E - 1)) * TH];
    }
};

template <typename T, int L, int E>
__device__ __forceinline__ cx<T> slope_fix_at(const SlopePhasors<T> &p, const Roots<T, L, E> &r) {
    return p.a0 + cmul(p.b1, r.rn) + cmulc(p.b2, r.r1) + cmul(p.b3, r.rm);
}

// Transforms of the two real sequences packed as p = c_0 + i c_M, from p and
// its conjugate mirror m = p[L - k]:  c_0 -> (p + conj m) / 2,
// c_M -> (p - conj m) / (2i).
template <typename T>
__device__ __forceinline__ cx<T> unpack_even(cx<T> p, cx<T> m) {
    return {T(0.5) * (p.x + m.x), T(0.5) * (p.y - m.y)};
}
template <typename T>
__device__ __forceinline__ cx<T> unpack_odd(cx<T> p, cx<T> m) {
    return {T(0.5) * (p.y + m.y), T(0.5) * (m.x - p.x)};
}

// Points per batch of spectrum loads in the multiply-accumulate of pass B,
// sized so that a batch's loads (six complex values per point) fit in the
// registers beside the transform data: 64 / E in FP32 (E <= 8: all E),
// 2 in FP64.
template <typename T, int E>
__host__ __device__ constexpr int mac_batch() { return sizeof(T) == 8 ? 2 : (E < 8 ? E : 64 / E); }

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
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = unit * G + gi;
    const bool valid = col < H;
    const int cl = valid ? col : 0;
    const bool packed = unit == 0;          // workgroup-uniform: the group holding column 0
    const bool is0 = packed && gi == 0;
    Lds<T> lds{buf, gi, G};

    // The column.  Only the first E/2 strided points of a thread can be data
    // rows (L >= 2 n_r); clamped, always valid addresses so the loads issue
    // back to back.
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int i = t + e * TH;
        v[e] = S[(size_t)(i < n_r ? i : n_r - 1) * H + cl];
    }
    // the four rows entering the slope correction, and the thread's phasors
    const cx<T> x0 = S[cl], x1 = S[(size_t)H + cl];
    const cx<T> xm2 = S[(size_t)(n_r - 2) * H + cl], xm1 = S[(size_t)(n_r - 1) * H + cl];
    const cx<T> wt = twL[t], wnt = twL[(int)(((unsigned)n_r * (unsigned)t) & (unsigned)(L - 1))];
    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (e >= E / 2 || !valid || i >= n_r) v[e] = cx<T>{T(0), T(0)};
    }
    fft_fwd<L, E, T>(v, t, lds, tw);
    if (packed) {   // column 0 reads the conjugate mirror points from LDS
#pragma unroll
        for (int e = 0; e < E; ++e) lds.st(t + e * TH, v[e]);
        __syncthreads();
    }

    const cx<T> *er = spec + (size_t)(0 * H + cl) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cl) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cl) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cl) * ldspec;
    const SlopeFix<T> a = slope_fix(x0, x1, xm2, xm1, ca, c0, cn);
    const SlopePhasors<T> ph = slope_phasors(a, wt, wnt);
    SlopePhasors<T> ph0 = ph, phM = ph;
    if (is0) {   // bins 0 and M of the packed column: real coefficients each
        ph0 = slope_phasors(slope_fix_part(a, false), wt, wnt);
        phM = slope_phasors(slope_fix_part(a, true), wt, wnt);
    }
    constexpr int CH = mac_batch<T, E>();
    cx<T> yr[E], yp[E];
#pragma unroll
    for (int cb = 0; cb < E; cb += CH) {
        // spectra of the batch issued together; column 0's slots 2, 3 hold
        // bin M's radial (even) spectra
        cx<T> sa[CH], sb[CH], sc[CH], sd[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int ku = t + (cb + j) * TH;
            sa[j] = spec_at<T, L>(er, ku, false);
            sb[j] = spec_at<T, L>(qr, ku, false);
            sc[j] = spec_at<T, L>(ep, ku, !is0);
            sd[j] = spec_at<T, L>(qp, ku, !is0);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = cb + j;
            const Roots<T, L, E> r(twL, n_r, e);
            if (is0) {
                const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                const cx<T> A = unpack_even(v[e], m), B = unpack_odd(v[e], m);
                const cx<T> f0 = slope_fix_at(ph0, r), fM = slope_fix_at(phM, r);
                const cx<T> y0 = cmul(sa[j], A) + cmul(sb[j], f0);
                const cx<T> yM = cmul(sc[j], B) + cmul(sd[j], fM);
                yr[e] = cx<T>{y0.x - yM.y, y0.y + yM.x};   // y0 + i yM
                yp[e] = cx<T>{T(0), T(0)};
            } else {
                const cx<T> f = slope_fix_at(ph, r);
                yr[e] = cmul(sa[j], v[e]) + cmul(sb[j], f);
                yp[e] = cmul(sc[j], v[e]) + cmul(sd[j], f);
            }
        }
    }
    if (packed) __syncthreads();
    fft_inv<L, E, T>(yr, t, lds, tw);
    fft_inv<L, E, T>(yp, t, lds, tw);
    if (valid) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + e * TH;
            if (i < n_r) {
                Zr[(size_t)i * H + col] = yr[e];
                Zp[(size_t)i * H + col] = yp[e];
            }
        }
    }
}

// Sum of x over the threads of each column of the workgroup (the G columns
// are interleaved lane by lane: column gi = thread % G); every thread gets
// its column's sum.  Within a wave the lanes of a column combine by lane
// exchange; across waves through the first n_grp * G * Q complex slots of
// buf.  The caller's previous LDS use must be fenced by a barrier.
template <typename T, int Q>
__device__ __forceinline__ void column_sums(cx<T> (&x)[Q], int G, cx<T> *__restrict__ buf) {
    const int nthr = blockDim.x;
    const int width = nthr < 64 ? nthr : 64;
    for (int off = G; off < width; off <<= 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            x[q].x += __shfl_xor(x[q].x, off);
            x[q].y += __shfl_xor(x[q].y, off);
        }
    }
    if (nthr > 64) {
        const int gi = threadIdx.x % G;
        // one partial per (group, column): per wave when G < 64 (every wave
        // then holds all G columns), per thread otherwise
        const bool wide = G >= 64;
        const int grp = wide ? (int)threadIdx.x / G : (int)(threadIdx.x >> 6);
        const int n_grp = wide ? nthr / G : nthr >> 6;
        if (wide || (int)(threadIdx.x & 63) < G) {
#pragma unroll
            for (int q = 0; q < Q; ++q) buf[(grp * G + gi) * Q + q] = x[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            cx<T> s = buf[gi * Q + q];
            for (int g = 1; g < n_grp; ++g) s = s + buf[(g * G + gi) * Q + q];
            x[q] = s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Pass B, transpose: correlate with the kernels (conjugate spectra), then
// the transposed slope: the transposed central difference is in E'; the
// four-row correction needs the inverse transform of R = conj(Q_r) V_r +
// conj(Q_p) V_p at rows 0, n-1, n and L-1 only, four sums over k.
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
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = unit * G + gi;
    const bool valid = col < H;
    const int cl = valid ? col : 0;
    const bool packed = unit == 0;
    const bool is0 = packed && gi == 0;
    Lds<T> lds{buf, gi, G};

    // clamped, always valid addresses so the loads issue back to back; only
    // the first E/2 points of a thread can be data rows (L >= 2 n_r)
    cx<T> va[E], vb[E];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int i = t + e * TH;
        const size_t o = (size_t)(i < n_r ? i : n_r - 1) * H + cl;
        va[e] = Vr[o];
        vb[e] = Vp[o];
    }
    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (e >= E / 2 || !valid || i >= n_r) {
            va[e] = cx<T>{T(0), T(0)};
            vb[e] = cx<T>{T(0), T(0)};
        }
    }
    fft_fwd<L, E, T>(va, t, lds, tw);
    fft_fwd<L, E, T>(vb, t, lds, tw);
    if (packed) {   // column 0 reads the conjugate mirror points from LDS
#pragma unroll
        for (int e = 0; e < E; ++e) lds.st(t + e * TH, va[e]);
        __syncthreads();
    }

    const cx<T> *er = spec + (size_t)(0 * H + cl) * ldspec;
    const cx<T> *qr = spec + (size_t)(1 * H + cl) * ldspec;
    const cx<T> *ep = spec + (size_t)(2 * H + cl) * ldspec;
    const cx<T> *qp = spec + (size_t)(3 * H + cl) * ldspec;
    // The unnormalised inverse transform of R at rows 0, L-1, n, n-1:
    //   w[0] = sum R, w[1] = sum R W^k, w[2] = sum R W^(-n k),
    //   w[3] = sum R W^(-(n-1) k),
    // summed per thread against the roots (W^(j k) = W^(j t) r(j e)) and
    // turned into the thread's share with its phasors afterwards.
    cx<T> w[4] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    constexpr int CH = mac_batch<T, E>();
#pragma unroll
    for (int cb = 0; cb < E; cb += CH) {
        cx<T> sa[CH], sb[CH], sc[CH], sd[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int ku = t + (cb + j) * TH;
            sa[j] = spec_at<T, L>(er, ku, false);
            sb[j] = spec_at<T, L>(qr, ku, false);
            sc[j] = spec_at<T, L>(ep, ku, !is0);
            sd[j] = spec_at<T, L>(qp, ku, !is0);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = cb + j;
            cx<T> x, r;
            if (is0) {
                // bins 0 and M of the packed column; V_p's bins 0 and M do
                // not enter (the azimuthal spectra vanish there)
                const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                const cx<T> A = unpack_even(va[e], m), B = unpack_odd(va[e], m);
                const cx<T> x0 = cmulc(A, sa[j]), xM = cmulc(B, sc[j]);
                const cx<T> r0 = cmulc(A, sb[j]), rM = cmulc(B, sd[j]);
                x = cx<T>{x0.x - xM.y, x0.y + xM.x};
                r = cx<T>{r0.x - rM.y, r0.y + rM.x};
            } else {
                x = cmulc(va[e], sa[j]) + cmulc(vb[e], sc[j]);   // conj(E'_r) V_r + conj(E'_p) V_p
                r = cmulc(va[e], sb[j]) + cmulc(vb[e], sd[j]);   // conj(Q_r) V_r + conj(Q_p) V_p
            }
            va[e] = x;
            const Roots<T, L, E> ro(twL, n_r, e);
            w[0] = w[0] + r;
            w[1] = w[1] + cmul(r, ro.r1);
            w[2] = w[2] + cmulc(r, ro.rn);
            w[3] = w[3] + cmulc(r, ro.rm);
        }
    }
    if (packed) __syncthreads();
    {
        const cx<T> wt = twL[t];
        const cx<T> wnt = twL[(int)(((unsigned)n_r * (unsigned)t) & (unsigned)(L - 1))];
        const cx<T> wmt = cmulc(wnt, wt);   // W^((n-1) t)
        w[1] = cmul(w[1], wt);
        w[2] = cmulc(w[2], wnt);
        w[3] = cmulc(w[3], wmt);
    }
    column_sums<T, 4>(w, G, buf);
    fft_inv<L, E, T>(va, t, lds, tw);
    if (valid) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + e * TH;
            if (i < n_r) {
                // transposed four-row correction
                cx<T> acc = va[e];
                if (i == 0) acc = acc - scale(w[0], c0) - scale(w[1], ca);
                if (i == 1) acc = acc + scale(w[0], c0 - ca);
                if (i == n_r - 2) acc = acc + scale(w[3], ca - cn);
                if (i == n_r - 1) acc = acc + scale(w[3], cn) + scale(w[2], ca);
                D[(size_t)i * H + col] = acc;
            }
        }
    }
}

}  // namespace pf
