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
// Layouts: S and D are row-major [n_r][M] complex, M = n_phi/2; the two
// force channels travel together as row-major [n_r][M] pairs (Zr, Zp) and
// (Vr, Vp), so one point of both is one 16-byte (FP32) access.  Spectra are
// [2][M][L/2+1] pairs, (E'_r, Q_r) then (E'_p, Q_p) -- for column 0 the
// radial pairs of bin 0 and of bin M -- column-contiguous, holding k_u in
// [0, L/2]; the rest follows from the kernels' symmetry in phi.
#pragma once
#include "fft_core.hpp"

namespace pf {

// Streaming (non-temporal) stores of one complex value or one pair, for the
// row passes' outputs, which the next pass reads from other XCDs: they go
// out to memory during the pass instead of staying dirty in the XCD's L2
// until the end of the kernel (forward step 32.6 to 31.7 us at 1024 x 2048).
template <typename T>
__device__ __forceinline__ void store_stream(cx<T> *p, cx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 x = {v.x, v.y};
    __builtin_nontemporal_store(x, reinterpret_cast<v2 *>(p));
}
template <typename T>
__device__ __forceinline__ void store_stream(cx2<T> *p, cx2<T> v) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    const v4 x = {v.a.x, v.a.y, v.b.x, v.b.y};
    __builtin_nontemporal_store(x, reinterpret_cast<v4 *>(p));
}

// ---------------------------------------------------------------------------
// FP32 scaling per grid.  The column transforms sum up to L N_phi values of
// the density, so in FP32 a density near 2^104 would overflow them (and one
// near 2^-110 would reach subnormal intermediates).  Each call therefore
// scales the grid by a power of two, 2^-e with e = floor(log2 max|sigma|):
//   pass A notes max|sigma| (as float bits, which order like the
//     magnitudes) in one of 64 words by atomic maximum, one atomic per
//     wave (the wave's maximum by lane exchanges first); the words sit 128
//     bytes apart (word w at g[32 w]), each in a cache line of its own, so
//     the atomics of the pass spread over 64 lines instead of queueing on
//     one;
//   pass B reads the 64 words, scales its column by 2^-e (after the first
//     stage of the column transform, which sums at most 8 values), stores
//     its output still scaled, and its first workgroup writes e to
//     g[32 * 64];
//   pass C reads e, multiplies its outputs by 2^e, and clears the 64 words
//     for the next call (pass B is done with them).
// Every pass of a call runs after the previous one on the stream.  Between
// the note and the final multiply every value is the unscaled one times
// 2^-e, so wherever the outputs are normal numbers they are bit for bit
// those of the unscaled computation times 2^e -- and no intermediate leaves
// the FP32 range as long as max|sigma| N_phi stays below 2^127.  For
// |e| <= kScaleFree the unscaled sums stay far inside the range (below
// 2^33 L N_phi <= 2^59 before the product with the kernel spectra), so e is
// taken as 0 there and the multiplies by 2^-e and 2^e are skipped (a
// branch on a value uniform over the workgroup).  FP64 is not scaled.
// ---------------------------------------------------------------------------
// (the layout constants kScale* are in fft_core.hpp)

// The maximum of m over a whole wave (all 64 lanes active), uniform (in a
// scalar register): row shifts by 1, 2, 4 and 8 lanes (lanes before a row's
// start read 0, the identity of the unsigned maximum) leave each row's
// maximum in its lane 15; the row broadcasts of lanes 15 and 31 carry them
// on to lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned m) {
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x111, 0xf, 0xf, false));
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x112, 0xf, 0xf, false));
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x114, 0xf, 0xf, false));
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x118, 0xf, 0xf, false));
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x142, 0xa, 0xf, false));
    m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)m, 63);
}

template <typename T, int E, int C>
__device__ __forceinline__ void scale_note(unsigned *__restrict__ g, const cx<T> (&v)[C][E]) {
    if constexpr (sizeof(T) == 4) {
        unsigned m = 0u;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < E; ++e)
                m = max(m, max(__float_as_uint(fabsf(v[c][e].x)), __float_as_uint(fabsf(v[c][e].y))));
        unsigned *const w = &g[((blockIdx.x * 8 + (threadIdx.x >> 6)) & (kScaleWords - 1)) * kScaleStride];
        if ((threadIdx.x | 63) < blockDim.x) {   // a whole wave: one atomic
            m = wave_max_u32(m);
            if ((threadIdx.x & 63) == 0) atomicMax(w, m);
        } else {   // the part-filled last wave of a small workgroup: every lane
            atomicMax(w, m);
        }
    }
}

// 2^-e and 2^e
template <typename T>
struct GridScale {
    T dn, up;
};
template <typename T>
__device__ __forceinline__ GridScale<T> scale_of(int ex) {
    return {__uint_as_float((unsigned)(127 - ex) << 23), __uint_as_float((unsigned)(127 + ex) << 23)};
}

// pass B: the first wave loads the 64 notes (lane i reads note i; issued
// before the column's loads) and reduces them while the first stage of the
// column transform runs; e (clamped to
// [-100, 100], 0 within [-kScaleFree, kScaleFree]) reaches the other waves
// through LDS across that stage's barrier, and the unit-0 workgroup writes
// it to g[kScaleE] for pass C.
// The column passes apply 2^-e after the first stage of their forward
// transforms (fft_fwd_zh_scaled).  FP32 passes always get the words; FP64
// passes are not scaled (ones).
template <typename T>
__device__ __forceinline__ unsigned scale_load(const unsigned *__restrict__ g) {
    if constexpr (sizeof(T) == 4)
        if (threadIdx.x < 64) return g[threadIdx.x * kScaleStride];
    return 0u;
}
__device__ __forceinline__ int &scale_slot() {
    __shared__ int s_ex;
    return s_ex;
}
// The scale step of the first column transform (the F of fft_stages): pre()
// in the first wave reduces the notes and publishes e, post() reads it.
template <typename T>
struct ScaleFind {
    unsigned *g;
    unsigned note;
    int unit;
    GridScale<T> *res;
    __device__ __forceinline__ void pre() const {
        if constexpr (sizeof(T) == 4) {
            if (threadIdx.x < 64) {
                const unsigned m = wave_max_u32(note);
                int ex = min(max((int)((m >> 23) & 0xffu) - 127, -100), 100);
                if (ex >= -kScaleFree && ex <= kScaleFree) ex = 0;
                if (threadIdx.x == 0) {
                    scale_slot() = ex;
                    if (unit == 0) g[kScaleE] = (unsigned)ex;
                }
            }
        }
    }
    __device__ __forceinline__ T post() const {
        if constexpr (sizeof(T) == 4) {
            *res = scale_of<T>(__builtin_amdgcn_readfirstlane(scale_slot()));
            return res->dn;
        }
        *res = GridScale<T>{T(1), T(1)};
        return T(1);
    }
};
// A scale already known (the second column transform of the adjoint).
template <typename T>
struct ScaleKnown {
    T s;
    __device__ __forceinline__ void pre() const {}
    __device__ __forceinline__ T post() const { return s; }
};

// pass C: e as pass B wrote it; the unit-0 workgroup of the grid clears
// the notes (any number of threads)
template <typename T>
__device__ __forceinline__ T scale_finish(unsigned *__restrict__ g, int unit) {
    if constexpr (sizeof(T) == 4) {
        const int ex = (int)g[kScaleE];
        if (unit == 0)
            for (int i = threadIdx.x; i < kScaleWords; i += blockDim.x) g[i * kScaleStride] = 0u;
        return scale_of<T>(ex).up;
    }
    return T(1);
}

// ---------------------------------------------------------------------------
// Row transforms along phi.  A real row of N = 2M points goes through one
// M-point complex transform of z[n] = x[2n] + i x[2n+1]; its spectrum is
// the packed half spectrum (bin 0 = (X_0, X_M)).  C = 1 or 2 channels: with
// C = 2 a thread holds the same points of two fields' rows (the two force
// channels), whose half spectra are stored as pairs.
// Workgroup: G rows x (M/E) threads; LDS buf: C*G*padded_len(M) complex.
// ---------------------------------------------------------------------------
template <typename T, int M, int E, int C>
__device__ __forceinline__ void row_lds(cx<T> *buf, int gi, int G, Lds<T> (&lds)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c)
        lds[c] = Lds<T>{buf + (size_t)c * G * padded_len(M), gi * padded_len(M), 1};
}

// Pass A: rows of in0 (and in1 for C = 2) -> packed half spectra
// (out: [n_rows][M] complex for C = 1, [n_rows][M] pairs for C = 2).
template <typename T, int M, int E, int C>
__device__ __forceinline__ void body_rows_r2c(int unit, int G, cx<T> *__restrict__ buf,
                                              const T *__restrict__ in0,
                                              const T *__restrict__ in1, int n_rows,
                                              cx<T> *__restrict__ out,
                                              const cx<T> *__restrict__ twN,
                                              unsigned *__restrict__ gscale = nullptr) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0
    Lds<T> lds[C];
    row_lds<T, M, E, C>(buf, gi, G, lds);

    // unconditional loads (in bounds for every lane) so they issue together
    cx<T> v[C][E];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<T> *xz = reinterpret_cast<const cx<T> *>((c == 0 ? in0 : in1) + (size_t)i * N);
#pragma unroll
        for (int e = 0; e < E; ++e) v[c][e] = xz[t + e * TH];
    }
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!active) v[c][e] = cx<T>{T(0), T(0)};
    scale_note<T, E, C>(gscale, v);
    fft_fwd<M, E, C, T>(v, t, lds, tw);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[c].st_split(lds_pad(t), e * TH, v[c][e]);
    __syncthreads();
    cx<T> o[C][E];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            const cx<T> zk = lds[c].ld(k), zm = lds[c].ld((M - k) & (M - 1));
            const cx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            // (zk - conj zm) / (2i)
            const cx<T> od = {T(0.5) * (zk.y + zm.y), -T(0.5) * (zk.x - zm.x)};
            cx<T> x = cmac(ev, twN[k], od);
            if (k == 0) x = cx<T>{zk.x + zk.y, zk.x - zk.y};   // (X_0, X_M), both real
            o[c][e] = x;
        }
    if (active) {
        if constexpr (C == 1) {
            cx<T> *orow = out + (size_t)i * M;
#pragma unroll
            for (int e = 0; e < E; ++e) store_stream(&orow[t + e * TH], o[0][e]);
        } else {
            cx2<T> *orow = reinterpret_cast<cx2<T> *>(out) + (size_t)i * M;
#pragma unroll
            for (int e = 0; e < E; ++e)
                store_stream(&orow[t + e * TH], cx2<T>{o[0][e], o[1][e]});
        }
    }
}

// Pass C: packed half rows (in: [n_rows][M] complex for C = 1, pairs for
// C = 2) -> real rows of out0 (and out1), unnormalised inverse.  turn in
// [0, N): the rows come out turned by that many points (out[j] is the
// inverse at j - turn), bin k taken times exp(-2 pi i k turn / N) -- the
// constant phase of a whole-cell shift in phi; 0 for no turn.
template <typename T, int M, int E, int C>
__device__ __forceinline__ void body_rows_c2r(int unit, int G, cx<T> *__restrict__ buf,
                                              const cx<T> *__restrict__ in, int n_rows,
                                              T *__restrict__ out0, T *__restrict__ out1,
                                              const cx<T> *__restrict__ twN,
                                              unsigned *__restrict__ gscale = nullptr,
                                              int turn = 0) {
    constexpr int TH = M / E;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0
    Lds<T> lds[C];
    row_lds<T, M, E, C>(buf, gi, G, lds);

    // unconditional loads (in bounds for every lane) so they issue together;
    // the mirror bins M - k come from LDS
    cx<T> xk[C][E], xm[C][E], wk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
        if constexpr (C == 1) {
            const cx<T> *X = in + (size_t)i * M;
            xk[0][e] = X[k];
        } else {
            const cx2<T> *X = reinterpret_cast<const cx2<T> *>(in) + (size_t)i * M;
            const cx2<T> a = X[k];
            xk[0][e] = a.a;
            xk[C - 1][e] = a.b;
        }
        wk[e] = twN[k];   // exp(-2 pi i k / N)
    }
    if (turn) {   // uniform
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            const cx<T> ph = twN[(k * turn) & (N - 1)];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (k == 0)   // packed (X_0, X_M): X_M times (-1)^turn
                    xk[c][e].y = (turn & 1) ? -xk[c][e].y : xk[c][e].y;
                else
                    xk[c][e] = cmul(xk[c][e], ph);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[c].st_split(lds_pad(t), e * TH, xk[c][e]);
    lds_barrier();
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) xm[c][e] = lds[c].ld((M - (t + e * TH)) & (M - 1));
    lds_barrier();
    Twiddles<M, E, T> tw;
    tw.load(t, twN, 2);
    if (t == 0) {   // unpack bin 0 = (X_0, X_M)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const cx<T> p = xk[c][0];
            xk[c][0] = cx<T>{p.x, T(0)};
            xm[c][0] = cx<T>{p.y, T(0)};
        }
    }
    cx<T> v[C][E];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cx<T> s = {xk[c][e].x + xm[c][e].x, xk[c][e].y - xm[c][e].y};   // X[k] + conj X[M-k]
            const cx<T> d = {xk[c][e].x - xm[c][e].x, xk[c][e].y + xm[c][e].y};   // X[k] - conj X[M-k]
            // s + i d exp(+2 pi i k / N): i conj(w) = (w.y, w.x) for w = wk
            const cx<T> iw = {wk[e].y, wk[e].x};
            v[c][e] = active ? cmac(s, d, iw) : cx<T>{T(0), T(0)};
        }
    fft_inv<M, E, C, T>(v, t, lds, tw);
    const T up = scale_finish<T>(gscale, unit);
    if (up != T(1))
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < E; ++e) v[c][e] = scale(v[c][e], up);
    if (active) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            cx<T> *yz = reinterpret_cast<cx<T> *>((c == 0 ? out0 : out1) + (size_t)i * N);
#pragma unroll
            for (int e = 0; e < E; ++e) store_stream(&yz[t + e * TH], v[c][e]);
        }
    }
}

// ---------------------------------------------------------------------------
// Spectrum access.  Spectra are stored for k_u in [0, L/2]; the kernels'
// symmetry in phi gives the rest: E_r, Q_r are even in n (the value at -k_u
// is the conjugate), E_p, Q_p odd (minus the conjugate).  Point e of thread
// t is k_u = t + e TH: for e < E/2 it is stored as is; for e > E/2 it is
// the mirror of L - k_u; for e = E/2 it is k_u = L/2 + t, stored at L/2 for
// t = 0 and the mirror of L/2 - t otherwise.  With e fixed by the unrolled
// loops the index is t plus a constant and the mirror's conjugation folds
// into the product (no branch, no sign flips).
// ---------------------------------------------------------------------------
template <int L, int E>
__device__ __forceinline__ int spec_index(int t, int e) {
    constexpr int TH = L / E;
    return e < E / 2 ? t + e * TH : L - t - e * TH;
}

// x S (CJ false) or x conj(S) (CJ true) for the spectrum value S of point
// e whose stored value is s (spec_index); ODD: a kernel odd in phi, whose
// mirror is -conj rather than conj.  t0: the thread is t = 0.  spec_mac adds
// the product to acc (fused).  The mirror's conjugation and sign fold into
// the operands: S = w with w = s, or the mirror of s.
template <typename T, int E, bool ODD>
__device__ __forceinline__ cx<T> spec_value(cx<T> s, int e, bool t0) {
    const cx<T> m = ODD ? cx<T>{-s.x, s.y} : cx<T>{s.x, -s.y};
    if (e == E / 2) return t0 ? s : m;
    return e < E / 2 ? s : m;
}

template <typename T, int E, bool ODD, bool CJ>
__device__ __forceinline__ cx<T> spec_mul(cx<T> s, cx<T> x, int e, bool t0) {
    const cx<T> w = spec_value<T, E, ODD>(s, e, t0);
    return CJ ? cx<T>{fmadd(x.x, w.x, x.y * w.y), fmadd(x.y, w.x, -(x.x * w.y))}
              : cx<T>{fmadd(x.x, w.x, -(x.y * w.y)), fmadd(x.x, w.y, x.y * w.x)};
}

template <typename T, int E, bool ODD, bool CJ>
__device__ __forceinline__ cx<T> spec_mac(cx<T> acc, cx<T> s, cx<T> x, int e, bool t0) {
    const cx<T> w = spec_value<T, E, ODD>(s, e, t0);
    return CJ ? cmacc(acc, x, w) : cmac(acc, x, w);
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
// W^(j e TH) = w^(j e), w = exp(-2 pi i / E) an E-th root of unity.  So per
// thread
//   b1 = an W^(n t),  b2 = am1 W^-t,  b3 = an1 W^((n-1) t)
// and per point, with w^(n e) the same for the whole workgroup (read from
// the table) and w^-e a constant of the unrolled code,
//   a0 + b2 w^-e + w^(n e) (b1 + b3 w^-e).
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

// w^(n e) for point e, read from the L-point table (w^q = W^(q L / E)) at an
// address that is the same for every lane
template <typename T, int L, int E>
__device__ __forceinline__ cx<T> root_ne(const cx<T> *__restrict__ twL, int n, int e) {
    return twL[((n * e) & (E - 1)) * (L / E)];
}

template <typename T, int E>
__device__ __forceinline__ cx<T> slope_fix_at(const SlopePhasors<T> &p, cx<T> rne, int e) {
    return cmac(mul_root_add<E>(p.a0, p.b2, -e), rne, mul_root_add<E>(p.b1, p.b3, -e));
}

// The boundary rows a correction reads: rows 0 .. SO-1 and n-SO .. n-1 of the
// column (SO = 2 for the four-row correction, 4 for the eight-row one).
template <typename T, int SO>
struct SlopeRows {
    cx<T> lo[SO], hi[SO];
};
template <typename T, int SO>
__device__ __forceinline__ SlopeRows<T, SO> slope_rows(const cx<T> *__restrict__ S, int H,
                                                       int n_r, int cl) {
    SlopeRows<T, SO> b;
#pragma unroll
    for (int q = 0; q < SO; ++q) b.lo[q] = S[(size_t)q * H + cl];
#pragma unroll
    for (int q = 0; q < SO; ++q) b.hi[q] = S[(size_t)(n_r - SO + q) * H + cl];
    return b;
}
template <typename T, int SO>
__device__ __forceinline__ SlopeRows<T, SO> scaled(SlopeRows<T, SO> b, T s) {
#pragma unroll
    for (int q = 0; q < SO; ++q) {
        b.lo[q] = scale(b.lo[q], s);
        b.hi[q] = scale(b.hi[q], s);
    }
    return b;
}

// Coefficients of the radial slope g = r delta^r on the logarithmic grid:
// ca three-point central, c0 and cn one-sided on the first and last rows,
// c4 five-point central (slope order 4 only).
template <typename T>
struct SlopeCoef {
    T ca, c0, cn, c4;
};

template <typename T>
__device__ __forceinline__ SlopeFix<T> slope_fix(const SlopeRows<T, 2> &b, const SlopeCoef<T> &k) {
    return slope_fix(b.lo[0], b.lo[1], b.hi[0], b.hi[1], k.ca, k.c0, k.cn);
}

// ---------------------------------------------------------------------------
// Eight-row correction of the radial slope of order 4.  The slope is the
// five-point difference c4 (c[i-2] - 8 c[i-1] + 8 c[i+1] - c[i+2]) on rows
// 2 .. n-3 (its circular form on the padded column is folded into the
// spectra as D(k) = 2i c4 (8 sin(2 pi k / L) - sin(4 pi k / L))), the
// three-point ca (c[i+1] - c[i-1]) on rows 1 and n-2 and the one-sided
// differences on rows 0 and n-1.  It differs from the circular five-point
// difference of the zero-padded column at eight rows (d_q = c[n-4+q]):
//   row 0      c0 (c1 - c0) - c4 (8 c1 - c2)
//   row 1      ca (c2 - c0) - c4 (8 (c2 - c0) - c3)
//   row n - 2  ca (d3 - d1) - c4 (8 (d3 - d1) + d0)
//   row n - 1  cn (d3 - d2) - c4 (d1 - 8 d2)
//   row n      c4 (8 d3 - d2)
//   row n + 1  -c4 d3
//   row L - 1  c4 (c1 - 8 c0)
//   row L - 2  c4 c0
// (n >= 4).  At k = t + e TH the rows j near 0 give a_j W^(j t) w^(j e) and
// those near n give w^(n e) a_j W^(j t) w^((j - n) e), as for four rows.
// ---------------------------------------------------------------------------
template <typename T>
struct SlopeFix4 {
    cx<T> a0, a1, am1, am2, an2, an1, an, anp1;
};

template <typename T>
__device__ __forceinline__ SlopeFix4<T> slope_fix(const SlopeRows<T, 4> &b, const SlopeCoef<T> &k) {
    const cx<T> *c = b.lo, *d = b.hi;
    SlopeFix4<T> s;
    s.a0 = scale(c[1] - c[0], k.c0) - scale(scale(c[1], T(8)) - c[2], k.c4);
    s.a1 = scale(c[2] - c[0], k.ca) - scale(scale(c[2] - c[0], T(8)) - c[3], k.c4);
    s.an2 = scale(d[3] - d[1], k.ca) - scale(scale(d[3] - d[1], T(8)) + d[0], k.c4);
    s.an1 = scale(d[3] - d[2], k.cn) - scale(d[1] - scale(d[2], T(8)), k.c4);
    s.an = scale(scale(d[3], T(8)) - d[2], k.c4);
    s.anp1 = scale(d[3], -k.c4);
    s.am1 = scale(c[1] - scale(c[0], T(8)), k.c4);
    s.am2 = scale(c[0], k.c4);
    return s;
}

template <typename T>
__device__ __forceinline__ SlopeFix4<T> slope_fix_part(const SlopeFix4<T> &s, bool imag) {
    auto pick = [imag](cx<T> a) { return cx<T>{imag ? a.y : a.x, T(0)}; };
    return {pick(s.a0), pick(s.a1),  pick(s.am1), pick(s.am2),
            pick(s.an2), pick(s.an1), pick(s.an),  pick(s.anp1)};
}

template <typename T>
struct SlopePhasors4 {
    cx<T> a0, l1, lm1, lm2, h0, h1, hm1, hm2;
};

template <typename T>
__device__ __forceinline__ SlopePhasors4<T> slope_phasors(const SlopeFix4<T> &s, cx<T> wt,
                                                          cx<T> wnt) {
    const cx<T> wtc = conj(wt), w2c = cmul(wtc, wtc);
    return {s.a0,
            cmul(s.a1, wt),
            cmul(s.am1, wtc),
            cmul(s.am2, w2c),
            cmul(s.an, wnt),
            cmul(s.anp1, cmul(wnt, wt)),
            cmul(s.an1, cmul(wnt, wtc)),
            cmul(s.an2, cmul(wnt, w2c))};
}

template <typename T, int E>
__device__ __forceinline__ cx<T> slope_fix_at(const SlopePhasors4<T> &p, cx<T> rne, int e) {
    const cx<T> lo =
        mul_root_add<E>(mul_root_add<E>(mul_root_add<E>(p.a0, p.l1, e), p.lm1, -e), p.lm2, -2 * e);
    const cx<T> hi =
        mul_root_add<E>(mul_root_add<E>(mul_root_add<E>(p.h0, p.h1, e), p.hm1, -e), p.hm2, -2 * e);
    return cmac(lo, rne, hi);
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

// Points per batch of spectrum loads when a column pass reads its spectra
// straight from global memory (kernels without the LDS prefetch): one pair
// per point and multiply-accumulate sweep, so that a batch's loads fit in
// the registers beside the transform data: 64 / E in FP32 (E <= 8: all E),
// two in FP64.
template <typename T, int E>
__host__ __device__ constexpr int mac_batch() {
    return sizeof(T) == 8 ? 2 : (E < 8 ? E : 64 / E);
}

// ---------------------------------------------------------------------------
// Pass B, forward.  Workgroup: G columns x (L/E) threads, lane -> (t, column)
// with the G columns interleaved (consecutive lanes read consecutive
// columns of a row).  LDS buf: G*padded_len(L) complex.
// S: [n_r][H] complex (the source rows); Z: [n_out][H] pairs (Zr, Zp), the
// destination rows; spec: [2][H][ldspec] pairs.
// ---------------------------------------------------------------------------
// Entries of one spectrum half per column in the LDS prefetch region:
// L/2 + 1 rounded up to whole 64-lane chunks and, when a column has at
// least 64 threads (L / E >= 64), to a multiple of L / E, so that every
// wave issues the same number of chunk loads, known at compile time.
template <int L, int E>
__host__ __device__ constexpr int spec_prefetch_len() {
    constexpr int Q = (L / E) > 64 ? (L / E) : 64;
    return ((L / 2 + 1) + Q - 1) / Q * Q;
}

// The spectrum pairs of one half (radial (E'_r, Q_r) at half = spec, or
// azimuthal (E'_p, Q_p) at half = spec + H ldspec) of the workgroup's G
// columns from global memory straight into LDS, spl[G][spec_prefetch_len<L,
// E>()] (a byte copy of the leading pairs of each column): buffer loads with
// the LDS-direct flag, 16 bytes per lane (half a pair in FP64), 1 KB per
// wave instruction, no registers held.  The caller waits (all counters 0,
// then a barrier) before reading.  With L / E >= 64 the G columns take
// G L / (64 E) waves and each wave issues LP U E / L chunk loads (U = 16-byte
// units per pair), a count fixed at compile time: the compiler can then wait
// for loads issued before these without waiting for these, and when spl is
// an LDS array of its own the transforms' LDS accesses do not wait for them
// either.  A chunk's address is the lane's 16-byte slot (one register for
// every chunk) plus a wave-uniform offset in a scalar register; the last
// chunk of a column may run past the column's L/2 + 1 pairs, into the next
// column or, for the last column, into the spectra's tail pad
// (kSpecTailPad), and those LDS slots are never read.  Offsets are 32-bit:
// one half of the spectra must be below 2 GB (checked by the host).
template <typename T, int L, int E>
__device__ __forceinline__ void prefetch_spectra(int unit, int G, int H, int ldspec,
                                                 const cx2<T> *__restrict__ half, cx2<T> *spl) {
    constexpr int U = (int)sizeof(cx2<T>) / 16;     // 16-byte units per pair
    static_assert(U == 1 || U == 2, "16- or 32-byte pairs");
    constexpr int LP = spec_prefetch_len<L, E>();
    constexpr int NCH = LP * U / 64;                // 64-lane chunks per column
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // whole waves (the shape check requires it); at least one, so the
    // wave-uniform loop below always advances
    const int nw = max(1, (int)(blockDim.x >> 6));
    // raw buffer over the half and the data beyond it up to the tail pad
    // (stride 0, byte offsets); the last word is the data-format field every
    // gfx9 raw buffer access uses
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<cx2<T> *>(half), (short)0, 2 * H * ldspec * 16 * U, 0x00020000);
    unsigned char *const dst = reinterpret_cast<unsigned char *>(spl);
    const int voff = lane * 16;
    auto chunk = [&](int c) {                       // c is wave-uniform
        const int g2 = c / NCH, q = c % NCH;
        const int cg = unit * G + g2;
        const int ccl = cg < H ? cg : 0;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs,
            (__attribute__((address_space(3))) void *)(dst + ((size_t)g2 * LP * U + q * 64) * 16),
            16, voff, (ccl * ldspec * U + q * 64) * 16, 0, 0);
    };
    if constexpr (L / E >= 64) {
        // nw = G L / (64 E) waves, G NCH chunks: LP U E / L chunks per wave
#pragma unroll
        for (int k = 0; k < LP * U / (L / E); ++k) chunk(wv + k * nw);
    } else {
        for (int c = wv; c < G * NCH; c += nw) chunk(c);   // wave-uniform loop
    }
}

// Waits for this wave's prefetch, then for every wave's (the chunks of a
// column come from several waves).
__device__ __forceinline__ void prefetch_wait() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// One multiply-accumulate sweep of the column pass over the thread's E
// points with the spectrum pairs (A, B) of one half:
//   y[e] = A(k) x[e] + B(k) f[e]   (CJ false), or
//   y[e] = conj A(k) x[e],  z[e] = conj B(k) x[e]   (CJ true, the transpose),
// ODD for the azimuthal half (odd in phi).  The pairs come from the LDS
// prefetch region sl (PF) or from global memory sg in batches.
//
// The forward sweep takes the slope correction at the points either from f
// (KEEP: formed once, kept in registers for both sweeps) or forms it from
// the phasors ph (FP64, where 16 more registers per point would spill).
template <typename T, int L, int E, bool ODD, bool PF, bool KEEP, typename PH>
__device__ __forceinline__ void mac_fwd(cx<T> (&y)[E], const cx<T> (&x)[E], const cx<T> (&f)[E],
                                        const PH &ph, const cx<T> *__restrict__ twL,
                                        int n_r, const cx2<T> *sl, const cx2<T> *__restrict__ sg,
                                        int t) {
    const bool t0 = t == 0;
    constexpr int CH = PF ? E : mac_batch<T, E>();
#pragma unroll
    for (int cb = 0; cb < E; cb += CH) {
        cx2<T> s[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int ix = spec_index<L, E>(t, cb + j);
            s[j] = PF ? sl[ix] : sg[ix];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = cb + j;
            const cx<T> fe = KEEP ? f[e] : slope_fix_at<T, E>(ph, root_ne<T, L, E>(twL, n_r, e), e);
            y[e] = spec_mac<T, E, ODD, false>(spec_mul<T, E, ODD, false>(s[j].a, x[e], e, t0),
                                              s[j].b, fe, e, t0);
        }
    }
}

template <typename T, int L, int E, bool ODD, bool PF, bool ACC>
__device__ __forceinline__ void mac_adj(cx<T> (&y)[E], cx<T> (&z)[E], const cx<T> (&x)[E],
                                        const cx2<T> *sl, const cx2<T> *__restrict__ sg, int t,
                                        bool skip = false) {
    const bool t0 = t == 0;
    constexpr int CH = PF ? E : mac_batch<T, E>();
#pragma unroll
    for (int cb = 0; cb < E; cb += CH) {
        cx2<T> s[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int ix = spec_index<L, E>(t, cb + j);
            s[j] = PF ? sl[ix] : sg[ix];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = cb + j;
            if constexpr (ACC) {
                const cx<T> a = spec_mac<T, E, ODD, true>(y[e], s[j].a, x[e], e, t0);
                const cx<T> b = spec_mac<T, E, ODD, true>(z[e], s[j].b, x[e], e, t0);
                y[e] = skip ? y[e] : a;
                z[e] = skip ? z[e] : b;
            } else {
                y[e] = spec_mul<T, E, ODD, true>(s[j].a, x[e], e, t0);
                z[e] = spec_mul<T, E, ODD, true>(s[j].b, x[e], e, t0);
            }
        }
    }
}

// The transpose's four sums of R against the roots at one point k of the
// thread: w[0] += r, w[1] += r W^k, w[2] += r W^(-n k), w[3] += r W^(-(n-1) k),
// with the thread's share of each root (W^(j t)) applied afterwards, so per
// point r w^e, r w^-(n e) and r w^-((n-1) e) (rne = w^(n e)).
template <typename T, int E>
__device__ __forceinline__ void accum_w(cx<T> (&w)[4], cx<T> r, cx<T> rne, int e) {
    const cx<T> q = cmulc(r, rne);
    w[0] = w[0] + r;
    w[1] = mul_root_add<E>(w[1], r, e);
    w[2] = w[2] + q;
    w[3] = mul_root_add<E>(w[3], q, e);
}
// The eight sums of the slope of order 4: the four above and rows 1, L-2,
// n-2 and n+1, w[4] += r W^-k, w[5] += r W^(2k), w[6] += r W^(-(n-2) k),
// w[7] += r W^(-(n+1) k).
template <typename T, int E>
__device__ __forceinline__ void accum_w(cx<T> (&w)[8], cx<T> r, cx<T> rne, int e) {
    const cx<T> q = cmulc(r, rne);
    w[0] = w[0] + r;
    w[1] = mul_root_add<E>(w[1], r, e);
    w[2] = w[2] + q;
    w[3] = mul_root_add<E>(w[3], q, e);
    w[4] = mul_root_add<E>(w[4], r, -e);
    w[5] = mul_root_add<E>(w[5], r, 2 * e);
    w[6] = mul_root_add<E>(w[6], q, 2 * e);
    w[7] = mul_root_add<E>(w[7], q, -e);
}

// The forward column transform of a zero-padded column, times the grid
// scale that f gives: in FP32 applied after the first stage, in FP64 not at
// all (f still runs, and gives one).
template <int L, int E, typename T, typename F>
__device__ __forceinline__ void fft_col_fwd(cx<T> (&v)[E], int t, const Lds<T> &lds,
                                            const Twiddles<L, E, T> &tw, F f) {
    if constexpr (sizeof(T) == 4) {
        fft_fwd_zh_scaled<L, E, T>(v, t, lds, tw, f);
    } else {
        f.pre();
        (void)f.post();
        fft_fwd<L, E, T, true>(v, t, lds, tw);
    }
}

// The column pass runs the two force channels one after the other: the
// radial channel's multiply-accumulate with the radial pairs, then, while
// its inverse transform runs, the azimuthal pairs arrive (in the LDS region
// the radial pairs held), then the azimuthal channel.  So the spectrum
// loads of the second half overlap a transform instead of waiting in the
// multiply-accumulate, and no point's work depends on a per-lane branch
// outside the one workgroup that holds the packed column 0.
// PF: the spectrum pairs go to LDS at spl (G spec_prefetch_len<L, E>()
// pairs), one half at a time.
// SO: order of the radial slope (2: the four-row correction; 4: five-point
// differences and the eight-row correction, c4 their coefficient).
template <typename T, int L, int E, bool PF = false, int SO = 2>
__device__ __forceinline__ void body_cols_fwd(int unit, int G, cx<T> *__restrict__ buf,
                                              const cx<T> *__restrict__ S,
                                              cx2<T> *__restrict__ Z,
                                              const cx2<T> *__restrict__ spec, int H, int n_r,
                                              int n_out, int ldspec, T ca, T c0, T cn,
                                              const cx<T> *__restrict__ twL,
                                              cx2<T> *spl = nullptr,
                                              unsigned *__restrict__ gscale = nullptr,
                                              T c4 = T(0)) {
    static_assert(SO == 2 || SO == 4, "slope order");
    constexpr int TH = L / E;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = unit * G + gi;
    const bool valid = col < H;
    const int cl = valid ? col : 0;
    const bool packed = unit == 0;          // workgroup-uniform: the group holding column 0
    const bool is0 = packed && gi == 0;
    const Lds<T> lds{buf, gi, G};
    constexpr int LP = spec_prefetch_len<L, E>();
    const cx2<T> *const srad = spec;                        // (E'_r, Q_r) per column
    const cx2<T> *const sazi = spec + (size_t)H * ldspec;   // (E'_p, Q_p) per column

    // The scale note first: loads complete in order, so the first wave's
    // wait for it (after the first transform stage) waits for no later load.
    const unsigned note = scale_load<T>(gscale);
    // The column.  Only the first E/2 strided points of a thread can be data
    // rows (L >= 2 n_r); clamped, always valid addresses so the loads issue
    // back to back.
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int i = t + e * TH;
        v[e] = S[(size_t)(i < n_r ? i : n_r - 1) * H + cl];
    }
    // the rows entering the slope correction, and the thread's phasors
    SlopeRows<T, SO> br = slope_rows<T, SO>(S, H, n_r, cl);
    const SlopeCoef<T> kf{ca, c0, cn, c4};
    const cx<T> wt = twL[t], wnt = twL[(int)(((unsigned)n_r * (unsigned)t) & (unsigned)(L - 1))];
    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
    // issued after the column's loads, which the transform waits for
    if constexpr (PF) prefetch_spectra<T, L, E>(unit, G, H, ldspec, srad, spl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (e >= E / 2 || !valid || i >= n_r) v[e] = cx<T>{T(0), T(0)};
    }
    GridScale<T> sc;
    fft_col_fwd<L, E, T>(v, t, lds, tw, ScaleFind<T>{gscale, note, unit, &sc});
    br = scaled(br, sc.dn);

    // FP32 (SPLIT): the radial channel's sweep and inverse transform, then
    // the azimuthal channel's (its spectrum pairs arriving meanwhile).  FP64:
    // one sweep forms both channels (radial pairs from LDS, azimuthal ones
    // from global memory), then the two inverse transforms -- fewer values
    // live across a transform (the split order spills at E = 8).
    constexpr bool SPLIT = sizeof(T) == 4;
    const auto ph = slope_phasors(slope_fix(br, kf), wt, wnt);
    const cx2<T> *sl = PF ? spl + (size_t)gi * LP : nullptr;
    const cx2<T> *const gr = srad + (size_t)cl * ldspec;
    const cx2<T> *const gp = sazi + (size_t)cl * ldspec;
    cx<T> y0[E], y1[E];
    if constexpr (SPLIT) {
        // transform of the slope correction at the thread's points, kept for
        // both sweeps with four rows; with eight rows (its phasors take twice
        // the registers) formed again in each sweep instead
        constexpr bool KEEPF = SO == 2;
        cx<T> f[E];
        if constexpr (KEEPF)
#pragma unroll
            for (int e = 0; e < E; ++e)
                f[e] = slope_fix_at<T, E>(ph, root_ne<T, L, E>(twL, n_r, e), e);

        // radial channel: y0 = E'_r X + Q_r B
        if constexpr (PF) prefetch_wait();
        mac_fwd<T, L, E, false, PF, KEEPF>(y0, v, f, ph, twL, n_r, sl, gr, t);
        if (packed) {
            // column 0 holds bins 0 and M packed as c_0 + i c_M: its radial
            // channel is y_0 + i y_M, from the bin-0 radial pairs (at the
            // radial place) and the bin-M radial pairs (at the azimuthal
            // place, read from global memory) applied to the two unpacked
            // transforms, which need the conjugate mirror points (through LDS)
#pragma unroll
            for (int e = 0; e < E; ++e) lds.st_split(lds_pad(t), e * TH, v[e]);
            lds_barrier();
            if (is0) {
                // the boundary rows again (read here rather than kept live
                // through the transform for this one column)
                const auto a = slope_fix(scaled(slope_rows<T, SO>(S, H, n_r, 0), sc.dn), kf);
                const auto ph0 = slope_phasors(slope_fix_part(a, false), wt, wnt);
                const auto phM = slope_phasors(slope_fix_part(a, true), wt, wnt);
                const bool t0 = t == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int ix = spec_index<L, E>(t, e);
                    const cx2<T> pr = PF ? sl[ix] : gr[ix];
                    const cx2<T> pm = gp[ix];
                    const cx<T> rne = root_ne<T, L, E>(twL, n_r, e);
                    const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                    const cx<T> A = unpack_even(v[e], m), B = unpack_odd(v[e], m);
                    const cx<T> f0 = slope_fix_at<T, E>(ph0, rne, e);
                    const cx<T> fM = slope_fix_at<T, E>(phM, rne, e);
                    const cx<T> ya = spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pr.a, A, e, t0), pr.b, f0, e, t0);
                    const cx<T> yb = spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pm.a, B, e, t0), pm.b, fM, e, t0);
                    y0[e] = cx<T>{ya.x - yb.y, ya.y + yb.x};   // ya + i yb
                }
            }
            lds_barrier();   // mirror reads done before the transforms reuse buf
        }
        if constexpr (PF) {
            // every wave has read its radial pairs: the azimuthal pairs go to
            // the same LDS region during the radial channel's inverse transform
            lds_barrier();
            prefetch_spectra<T, L, E>(unit, G, H, ldspec, sazi, spl);
        }
        fft_inv<L, E, T>(y0, t, lds, tw);

        // azimuthal channel: y1 = E'_p X + Q_p B (zero for column 0: the
        // azimuthal spectra vanish at bins 0 and M)
        if constexpr (PF) prefetch_wait();
        mac_fwd<T, L, E, true, PF, KEEPF>(y1, v, f, ph, twL, n_r, sl, gp, t);
#pragma unroll
        for (int e = 0; e < E; ++e) y1[e] = is0 ? cx<T>{T(0), T(0)} : y1[e];
        fft_inv<L, E, T>(y1, t, lds, tw);
    } else {
        if (packed) {   // column 0 reads the conjugate mirror points from LDS
#pragma unroll
            for (int e = 0; e < E; ++e) lds.st_split(lds_pad(t), e * TH, v[e]);
            lds_barrier();
        }
        // ph0 serves every column (ph is not kept beside it): the packed
        // column's lanes replace it and phM by the two bins' phasors
        auto ph0 = ph, phM = ph;
        if (is0) {   // bins 0 and M of the packed column: real coefficients each
            const auto a = slope_fix(scaled(slope_rows<T, SO>(S, H, n_r, 0), sc.dn), kf);
            ph0 = slope_phasors(slope_fix_part(a, false), wt, wnt);
            phM = slope_phasors(slope_fix_part(a, true), wt, wnt);
        }
        if constexpr (PF) prefetch_wait();
        constexpr int CH = mac_batch<T, E>();
        const bool t0 = t == 0;
#pragma unroll
        for (int cb = 0; cb < E; cb += CH) {
            // spectra of the batch issued together; column 0's azimuthal
            // place holds bin M's radial (even) pairs
            cx2<T> pr[CH], pp[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int ix = spec_index<L, E>(t, cb + j);
                pr[j] = PF ? sl[ix] : gr[ix];
                pp[j] = gp[ix];
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int e = cb + j;
                const cx<T> rne = root_ne<T, L, E>(twL, n_r, e);
                if (is0) {
                    const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                    const cx<T> A = unpack_even(v[e], m), B = unpack_odd(v[e], m);
                    const cx<T> f0 = slope_fix_at<T, E>(ph0, rne, e);
                    const cx<T> fM = slope_fix_at<T, E>(phM, rne, e);
                    const cx<T> ya = spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pr[j].a, A, e, t0), pr[j].b, f0, e, t0);
                    const cx<T> yb = spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pp[j].a, B, e, t0), pp[j].b, fM, e, t0);
                    y0[e] = cx<T>{ya.x - yb.y, ya.y + yb.x};   // ya + i yb
                    y1[e] = cx<T>{T(0), T(0)};
                } else {
                    const cx<T> f = slope_fix_at<T, E>(ph0, rne, e);
                    y0[e] = spec_mac<T, E, false, false>(
                        spec_mul<T, E, false, false>(pr[j].a, v[e], e, t0), pr[j].b, f, e, t0);
                    y1[e] = spec_mac<T, E, true, false>(
                        spec_mul<T, E, true, false>(pp[j].a, v[e], e, t0), pp[j].b, f, e, t0);
                }
            }
        }
        if (packed) lds_barrier();   // mirror reads done before the transforms reuse buf
        fft_inv<L, E, T>(y0, t, lds, tw);
        fft_inv<L, E, T>(y1, t, lds, tw);
    }
    if (valid) {
        // only the first E/2 points of a thread can be rows (L >= 2 n_out): the
        // rest of the last stage is never formed
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int i = t + e * TH;
            if (i < n_out) Z[(size_t)i * H + col] = cx2<T>{y0[e], y1[e]};   // still scaled
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
// V: [n_v][H] pairs (Vr, Vp) (the destination rows; n_v = n_r for one
// grid); D: [n_r][H] complex (the source rows, whose slopes the correction
// differences).  LDS buf: G*padded_len(L)
// complex.  As the forward pass, one spectrum half at a time: the radial
// pairs meet V_r's transform, and the azimuthal pairs arrive while V_p is
// transformed.
// PF: the spectrum pairs go to LDS at spl (G spec_prefetch_len<L, E>()
// pairs), one half at a time.
// ---------------------------------------------------------------------------
// SO: order of the radial slope, as for the forward pass (4: eight sums
// and the transposed eight-row correction).
template <typename T, int L, int E, bool PF = false, int SO = 2>
__device__ __forceinline__ void body_cols_adj(int unit, int G, cx<T> *__restrict__ buf,
                                              const cx2<T> *__restrict__ V,
                                              cx<T> *__restrict__ D,
                                              const cx2<T> *__restrict__ spec, int H, int n_r,
                                              int ldspec, T ca, T c0, T cn,
                                              const cx<T> *__restrict__ twL,
                                              cx2<T> *spl = nullptr,
                                              unsigned *__restrict__ gscale = nullptr,
                                              T c4 = T(0), int n_v = 0) {
    static_assert(SO == 2 || SO == 4, "slope order");
    constexpr int NW = SO == 4 ? 8 : 4;
    if (n_v <= 0) n_v = n_r;
    constexpr int TH = L / E;
    const int gi = threadIdx.x % G, t = threadIdx.x / G;
    const int col = unit * G + gi;
    const bool valid = col < H;
    const int cl = valid ? col : 0;
    const bool packed = unit == 0;
    const bool is0 = packed && gi == 0;
    const Lds<T> lds{buf, gi, G};
    constexpr int LP = spec_prefetch_len<L, E>();
    const cx2<T> *const srad = spec;
    const cx2<T> *const sazi = spec + (size_t)H * ldspec;

    // The scale note first: loads complete in order, so the first wave's
    // wait for it (after the first transform stage) waits for no later load.
    const unsigned note = scale_load<T>(gscale);
    // clamped, always valid addresses so the loads issue back to back; only
    // the first E/2 points of a thread can be data rows (L >= 2 n_v)
    cx<T> va[2][E];   // va[0]: V_r, va[1]: V_p
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int i = t + e * TH;
        const cx2<T> q = V[(size_t)(i < n_v ? i : n_v - 1) * H + cl];
        va[0][e] = q.a;
        va[1][e] = q.b;
    }
    Twiddles<L, E, T> tw;
    tw.load(t, twL, 1);
    // issued after the column's loads, which the transforms wait for
    if constexpr (PF) prefetch_spectra<T, L, E>(unit, G, H, ldspec, srad, spl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + e * TH;
        if (e >= E / 2 || !valid || i >= n_v) {
            va[0][e] = cx<T>{T(0), T(0)};
            va[1][e] = cx<T>{T(0), T(0)};
        }
    }
    GridScale<T> sc;
    // FP32 (SPLIT): V_r is transformed, meets the radial pairs, then V_p is
    // transformed while the azimuthal pairs arrive in LDS.  FP64: both
    // channels are transformed while the radial pairs arrive, then one
    // sweep takes the radial pairs from LDS and the azimuthal ones from
    // global memory, R entering the four sums point by point and the
    // transposed correlation replacing V_r in place (in FP64 the split order
    // keeps too many values live across a transform and spills).
    constexpr bool SPLIT = sizeof(T) == 4;
    const cx2<T> *sl = PF ? spl + (size_t)gi * LP : nullptr;
    const cx2<T> *const gr = srad + (size_t)cl * ldspec;
    const cx2<T> *const gp = sazi + (size_t)cl * ldspec;
    // The unnormalised inverse transform of R at rows 0, L-1, n, n-1:
    //   w[0] = sum R, w[1] = sum R W^k, w[2] = sum R W^(-n k),
    //   w[3] = sum R W^(-(n-1) k),
    // summed per thread against the roots (W^(j k) = W^(j t) r(j e)) and
    // turned into the thread's share with its phasors afterwards.
    cx<T> w[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) w[q] = cx<T>{T(0), T(0)};
    cx<T> xe[E];
    fft_col_fwd<L, E, T>(va[0], t, lds, tw, ScaleFind<T>{gscale, note, unit, &sc});
    if constexpr (SPLIT) {
        // radial half: xe = conj(E'_r) V_r, r = conj(Q_r) V_r
        if constexpr (PF) prefetch_wait();
        cx<T> r[E];
        mac_adj<T, L, E, false, PF, false>(xe, r, va[0], sl, gr, t);
        if (packed) {
            // bins 0 and M of the packed column 0, from the unpacked
            // transforms of V_r (conjugate mirror points through LDS) and
            // the bin-0 and bin-M radial pairs; V_p's bins 0 and M do not
            // enter (the azimuthal spectra vanish there)
#pragma unroll
            for (int e = 0; e < E; ++e) lds.st_split(lds_pad(t), e * TH, va[0][e]);
            lds_barrier();
            if (is0) {
                const bool t0 = t == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int ix = spec_index<L, E>(t, e);
                    const cx2<T> pr = PF ? sl[ix] : gr[ix];
                    const cx2<T> pm = gp[ix];
                    const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                    const cx<T> A = unpack_even(va[0][e], m), B = unpack_odd(va[0][e], m);
                    const cx<T> x0 = spec_mul<T, E, false, true>(pr.a, A, e, t0);
                    const cx<T> xM = spec_mul<T, E, false, true>(pm.a, B, e, t0);
                    const cx<T> r0 = spec_mul<T, E, false, true>(pr.b, A, e, t0);
                    const cx<T> rM = spec_mul<T, E, false, true>(pm.b, B, e, t0);
                    xe[e] = cx<T>{x0.x - xM.y, x0.y + xM.x};
                    r[e] = cx<T>{r0.x - rM.y, r0.y + rM.x};
                }
            }
            lds_barrier();   // mirror reads done before the transform reuses buf
        }
        if constexpr (PF) {
            // every wave has read its radial pairs: the azimuthal pairs go to
            // the same LDS region while V_p is transformed
            lds_barrier();
            prefetch_spectra<T, L, E>(unit, G, H, ldspec, sazi, spl);
        }
        fft_col_fwd<L, E, T>(va[1], t, lds, tw, ScaleKnown<T>{sc.dn});
        // azimuthal half: xe += conj(E'_p) V_p, r += conj(Q_p) V_p
        if constexpr (PF) prefetch_wait();
        mac_adj<T, L, E, true, PF, true>(xe, r, va[1], sl, gp, t, is0);
#pragma unroll
        for (int e = 0; e < E; ++e) accum_w<T, E>(w, r[e], root_ne<T, L, E>(twL, n_r, e), e);
    } else {
        fft_col_fwd<L, E, T>(va[1], t, lds, tw, ScaleKnown<T>{sc.dn});
        if (packed) {   // column 0 reads the conjugate mirror points from LDS
#pragma unroll
            for (int e = 0; e < E; ++e) lds.st_split(lds_pad(t), e * TH, va[0][e]);
            lds_barrier();
        }
        if constexpr (PF) prefetch_wait();
        constexpr int CH = mac_batch<T, E>();
        const bool t0 = t == 0;
#pragma unroll
        for (int cb = 0; cb < E; cb += CH) {
            cx2<T> pr[CH], pp[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int ix = spec_index<L, E>(t, cb + j);
                pr[j] = PF ? sl[ix] : gr[ix];
                pp[j] = gp[ix];
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int e = cb + j;
                cx<T> x, r;
                if (is0) {
                    // bins 0 and M of the packed column (bin M's radial pairs
                    // at the azimuthal place); V_p's bins 0 and M do not enter
                    const cx<T> m = lds.ld((L - (t + e * TH)) & (L - 1));
                    const cx<T> A = unpack_even(va[0][e], m), B = unpack_odd(va[0][e], m);
                    const cx<T> x0 = spec_mul<T, E, false, true>(pr[j].a, A, e, t0);
                    const cx<T> xM = spec_mul<T, E, false, true>(pp[j].a, B, e, t0);
                    const cx<T> r0 = spec_mul<T, E, false, true>(pr[j].b, A, e, t0);
                    const cx<T> rM = spec_mul<T, E, false, true>(pp[j].b, B, e, t0);
                    x = cx<T>{x0.x - xM.y, x0.y + xM.x};
                    r = cx<T>{r0.x - rM.y, r0.y + rM.x};
                } else {
                    // conj(E'_r) V_r + conj(E'_p) V_p, conj(Q_r) V_r + conj(Q_p) V_p
                    x = spec_mac<T, E, true, true>(
                        spec_mul<T, E, false, true>(pr[j].a, va[0][e], e, t0), pp[j].a,
                        va[1][e], e, t0);
                    r = spec_mac<T, E, true, true>(
                        spec_mul<T, E, false, true>(pr[j].b, va[0][e], e, t0), pp[j].b,
                        va[1][e], e, t0);
                }
                xe[e] = x;
                accum_w<T, E>(w, r, root_ne<T, L, E>(twL, n_r, e), e);
            }
        }
        if (packed) lds_barrier();   // mirror reads done before buf is reused
    }
    {
        const cx<T> wt = twL[t];
        const cx<T> wnt = twL[(int)(((unsigned)n_r * (unsigned)t) & (unsigned)(L - 1))];
        const cx<T> wmt = cmulc(wnt, wt);   // W^((n-1) t)
        w[1] = cmul(w[1], wt);
        w[2] = cmulc(w[2], wnt);
        w[3] = cmulc(w[3], wmt);
        if constexpr (SO == 4) {
            w[4] = cmulc(w[4], wt);                              // W^-t
            w[5] = cmul(w[5], cmul(wt, wt));                     // W^(2t)
            w[6] = cmulc(w[6], cmulc(wmt, wt));                  // W^(-(n-2) t)
            w[7] = cmulc(w[7], cmul(wnt, wt));                   // W^(-(n+1) t)
        }
    }
    column_sums<T, NW>(w, G, buf);
    fft_inv<L, E, T>(xe, t, lds, tw);
    if (valid) {
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {   // rows lie in the first half (L >= 2 n_r)
            const int i = t + e * TH;
            if (i < n_r) {
                cx<T> acc = xe[e];
                if constexpr (SO == 2) {   // transposed four-row correction
                    if (i == 0) acc = acc - scale(w[0], c0) - scale(w[1], ca);
                    if (i == 1) acc = acc + scale(w[0], c0 - ca);
                    if (i == n_r - 2) acc = acc + scale(w[3], ca - cn);
                    if (i == n_r - 1) acc = acc + scale(w[3], cn) + scale(w[2], ca);
                } else {
                    // transposed eight-row correction: the sums at rows
                    // 0, L-1, n, n-1, 1, L-2, n-2, n+1 (w[0..7]) back onto
                    // the boundary rows each correction row reads
                    const T k8 = T(8) * c4;
                    if (i == 0)
                        acc = acc - scale(w[0], c0) + scale(w[4], k8 - ca) - scale(w[1], k8) +
                              scale(w[5], c4);
                    if (i == 1) acc = acc + scale(w[0], c0 - k8) + scale(w[1], c4);
                    if (i == 2) acc = acc + scale(w[0], c4) + scale(w[4], ca - k8);
                    if (i == 3) acc = acc + scale(w[4], c4);
                    if (i == n_r - 4) acc = acc - scale(w[6], c4);
                    if (i == n_r - 3) acc = acc + scale(w[6], k8 - ca) - scale(w[3], c4);
                    if (i == n_r - 2) acc = acc + scale(w[3], k8 - cn) - scale(w[2], c4);
                    if (i == n_r - 1)
                        acc = acc + scale(w[6], ca - k8) + scale(w[3], cn) + scale(w[2], k8) -
                              scale(w[7], c4);
                }
                D[(size_t)i * H + col] = acc;   // still scaled
            }
        }
    }
}

}  // namespace pf
