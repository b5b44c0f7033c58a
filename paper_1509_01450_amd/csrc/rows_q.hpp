// rows_q.hpp -- the device bodies of the row transforms along phi for
// N_phi = 2 Q P (Q = 3 or 9, P a power of two), used by the standalone row
// kernels (pf_rows3.hip) and the batched row kernels (pf_batched.hip).
//
// A real row of N = 2 M points, M = Q P, goes through the M-point complex
// transform of z[m] = x[2m] + i x[2m+1], as in the power-of-two rows; that
// transform is split by decimation in time into Q P-point transforms Y_r
// of z[Qn + r] (r in [0, Q)), run by the power-of-two stages of fft_core.hpp
// as Q C transforms held together, and one radix-Q step in registers:
//   Z[k + jP] = sum_r (W_M^(r k) Y_r[k]) W_Q^(r j),   k in [0, P), j in [0, Q),
// W_M = exp(-2 pi i / M) (a radix-9 step as two radix-3 steps with the
// twiddles W_9^(n2 k1) between them).  Thread t holds the points
// k = t + e TH (TH = P / E) of all Q sub-transforms, so it forms Z at
// k + jP itself.  The packed half spectrum (bin 0 = (X_0, X_M)) then follows
// from Z and its mirror bins M - k as in the power-of-two rows.  The
// inverse (pass C) runs the same steps backwards:
//   z[Qn + r] = sum_k' W_P^(-n k') [W_M^(-r k') sum_j Z[k' + jP] W_Q^(-r j)].
// Workgroup: G rows x TH threads; LDS: C G rowq_len(P, Q) complex, per
// channel and row the Q P-point regions, reused for the mirror exchange.
#pragma once

#include "pass_bodies.hpp"

namespace pf {

// LDS slots per row and channel: Q padded P-point regions, or one padded
// QP-point region for the mirror exchange, whichever is longer
__host__ __device__ constexpr int rowq_len(int P, int Q) {
    return Q * padded_len(P) > padded_len(Q * P) ? Q * padded_len(P) : padded_len(Q * P);
}

// sqrt(3) / 2
template <typename T>
__device__ __forceinline__ T half_sqrt3() {
    return T(0.86602540378443864676372317075293618);
}

// y_j = sum_r a_r W_3^(s r j), s = -1 (forward) or +1 (inverse)
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cx<T> a0, cx<T> a1, cx<T> a2, cx<T> &y0, cx<T> &y1,
                                     cx<T> &y2) {
    const cx<T> s = a1 + a2, d = a1 - a2;
    const cx<T> m = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
    const T h = half_sqrt3<T>();
    // forward: W_3 = -1/2 - i sqrt(3)/2, so y1 = m - i h d; inverse: m + i h d
    const cx<T> ihd = INV ? cx<T>{-h * d.y, h * d.x} : cx<T>{h * d.y, -h * d.x};
    y0 = a0 + s;
    y1 = m + ihd;
    y2 = m - ihd;
}

// In place: a_j <- sum_r a_r W_Q^(s r j) (s = -1 forward, +1 inverse).
// w9[m] = W_9^m for m = 1, 2, 4 (Q = 9 only).  Q = 9: r = 3 n1 + n2 and
// j = k1 + 3 k2; the three-point transforms over n1, the twiddles
// W_9^(n2 k1), the three-point transforms over n2.
template <typename T, int Q, bool INV>
__device__ __forceinline__ void dftq(cx<T> (&a)[Q], const cx<T> (&w9)[5]) {
    if constexpr (Q == 3) {
        cx<T> y0, y1, y2;
        dft3<T, INV>(a[0], a[1], a[2], y0, y1, y2);
        a[0] = y0;
        a[1] = y1;
        a[2] = y2;
    } else {
        static_assert(Q == 9, "radix 3 or 9");
        cx<T> b[3][3];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2)
            dft3<T, INV>(a[n2], a[3 + n2], a[6 + n2], b[n2][0], b[n2][1], b[n2][2]);
#pragma unroll
        for (int n2 = 1; n2 < 3; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < 3; ++k1)
                b[n2][k1] = INV ? cmulc(b[n2][k1], w9[n2 * k1]) : cmul(b[n2][k1], w9[n2 * k1]);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1)
            dft3<T, INV>(b[0][k1], b[1][k1], b[2][k1], a[k1], a[k1 + 3], a[k1 + 6]);
    }
}

// W_9^m = exp(-2 pi i m / 9) from the N-point table (N = 18 P): twN[2 P m]
template <typename T, int P, int Q>
__device__ __forceinline__ void load_w9(const cx<T> *__restrict__ twN, cx<T> (&w9)[5]) {
#pragma unroll
    for (int m = 0; m < 5; ++m) w9[m] = cx<T>{T(1), T(0)};
    if constexpr (Q == 9) {
        w9[1] = twN[2 * P];
        w9[2] = twN[4 * P];
        w9[4] = twN[8 * P];
    }
}

template <typename T, int P, int Q, int C>
__device__ __forceinline__ void rowq_sub_lds(cx<T> *buf, int gi, int G, Lds<T> (&lds)[Q * C]) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < Q; ++r)
            lds[Q * c + r] = Lds<T>{buf, (c * G + gi) * rowq_len(P, Q) + r * padded_len(P), 1};
}

template <typename T, int P, int Q>
__device__ __forceinline__ Lds<T> rowq_mirror_lds(cx<T> *buf, int gi, int G, int c) {
    return Lds<T>{buf, (c * G + gi) * rowq_len(P, Q), 1};
}

// Pass A: rows of in0 (and in1 for C = 2) -> packed half spectra
// (out: [n_rows][M] complex for C = 1, pairs for C = 2).
template <typename T, int P, int Q, int E, int C>
__device__ __forceinline__ void body_rows_r2cq(int unit, int G, cx<T> *__restrict__ buf,
                                               const T *__restrict__ in0,
                                               const T *__restrict__ in1, int n_rows,
                                               cx<T> *__restrict__ out,
                                               const cx<T> *__restrict__ twN,
                                               unsigned *__restrict__ gscale) {
    constexpr int TH = P / E;
    constexpr int M = Q * P;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0
    Lds<T> lds[Q * C];
    rowq_sub_lds<T, P, Q, C>(buf, gi, G, lds);

    // z[Qn + r] for n = t + e TH: Q neighbouring complex values
    cx<T> v[Q * C][E];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<T> *xz = reinterpret_cast<const cx<T> *>((c == 0 ? in0 : in1) + (size_t)i * N);
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int r = 0; r < Q; ++r) v[Q * c + r][e] = xz[Q * (t + e * TH) + r];
    }
    Twiddles<P, E, T> tw;
    tw.load(t, twN, 2 * Q);   // the P-point table inside the N-point one
    cx<T> w9[5];
    load_w9<T, P, Q>(twN, w9);
#pragma unroll
    for (int a = 0; a < Q * C; ++a)
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!active) v[a][e] = cx<T>{T(0), T(0)};
    scale_note<T, E, Q * C>(gscale, v);
    fft_fwd<P, E, Q * C, T>(v, t, lds, tw);

    // the radix-Q step: Z at k + jP in place of Y_j
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            cx<T> a[Q];
            a[0] = v[Q * c][e];
#pragma unroll
            for (int r = 1; r < Q; ++r) a[r] = cmul(v[Q * c + r][e], twN[2 * r * k]);   // W_M^(rk)
            dftq<T, Q, false>(a, w9);
#pragma unroll
            for (int j = 0; j < Q; ++j) v[Q * c + j][e] = a[j];
        }
    }
    // mirror bins through LDS (the transforms' last reads are behind their
    // final barrier; a one-stage transform read nothing)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) mir.st(t + e * TH + j * P, v[Q * c + j][e]);
    }
    __syncthreads();
    // the packed half spectrum, in place
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                const cx<T> zk = v[Q * c + j][e], zm = mir.ld(k == 0 ? 0 : M - k);
                const cx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
                // (zk - conj zm) / (2i)
                const cx<T> od = {T(0.5) * (zk.y + zm.y), -T(0.5) * (zk.x - zm.x)};
                cx<T> x = cmac(ev, twN[k], od);
                if (k == 0) x = cx<T>{zk.x + zk.y, zk.x - zk.y};   // (X_0, X_M), both real
                v[Q * c + j][e] = x;
            }
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                if constexpr (C == 1) {
                    store_stream(&out[(size_t)i * M + k], v[j][e]);
                } else {
                    cx2<T> *orow = reinterpret_cast<cx2<T> *>(out) + (size_t)i * M;
                    store_stream(&orow[k], cx2<T>{v[j][e], v[Q + j][e]});
                }
            }
    }
}

// Pass C: packed half rows -> real rows of out0 (and out1), unnormalised
// inverse; turn in [0, N) turns the rows by that many points (bin k times
// exp(-2 pi i k turn / N)), as the power-of-two rows.
template <typename T, int P, int Q, int E, int C>
__device__ __forceinline__ void body_rows_c2rq(int unit, int G, cx<T> *__restrict__ buf,
                                               const cx<T> *__restrict__ in, int n_rows,
                                               T *__restrict__ out0, T *__restrict__ out1,
                                               const cx<T> *__restrict__ twN,
                                               unsigned *__restrict__ gscale, int turn) {
    constexpr int TH = P / E;
    constexpr int M = Q * P;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0

    // bins k = t + e TH + j P of channel c at v[Qc + j][e]
    cx<T> v[Q * C][E];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH + j * P;
            if constexpr (C == 1) {
                v[j][e] = in[(size_t)i * M + k];
            } else {
                const cx2<T> a = reinterpret_cast<const cx2<T> *>(in)[(size_t)i * M + k];
                v[j][e] = a.a;
                v[Q + j][e] = a.b;
            }
        }
    if (turn) {   // uniform
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                const cx<T> ph = twN[(k * turn) % N];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    cx<T> &x = v[Q * c + j][e];
                    if (k == 0)   // packed (X_0, X_M): X_M times (-1)^turn
                        x.y = (turn & 1) ? -x.y : x.y;
                    else
                        x = cmul(x, ph);
                }
            }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) mir.st(t + e * TH + j * P, v[Q * c + j][e]);
    }
    __syncthreads();
    cx<T> w9[5];
    load_w9<T, P, Q>(twN, w9);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
        // Z[k] of the complex transform, in place
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                cx<T> a = v[Q * c + j][e], m = mir.ld(k == 0 ? 0 : M - k);
                if (k == 0) {   // unpack bin 0 = (X_0, X_M)
                    m = cx<T>{a.y, T(0)};
                    a = cx<T>{a.x, T(0)};
                }
                const cx<T> s = {a.x + m.x, a.y - m.y};   // X[k] + conj X[M-k]
                const cx<T> d = {a.x - m.x, a.y + m.y};   // X[k] - conj X[M-k]
                const cx<T> w = twN[k];
                const cx<T> iw = {w.y, w.x};   // s + i d exp(+2 pi i k / N)
                v[Q * c + j][e] = cmac(s, d, iw);
            }
        // the inverse radix-Q step: U_r[k'] = W_M^(-r k') sum_j Z[k' + jP] W_Q^(-r j),
        // in place of Z at k' + rP
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            cx<T> a[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) a[j] = v[Q * c + j][e];
            dftq<T, Q, true>(a, w9);
            v[Q * c][e] = a[0];
#pragma unroll
            for (int r = 1; r < Q; ++r) v[Q * c + r][e] = cmulc(a[r], twN[2 * r * k]);
        }
    }
    __syncthreads();   // mirror reads done before the transforms reuse buf
    Lds<T> lds[Q * C];
    rowq_sub_lds<T, P, Q, C>(buf, gi, G, lds);
    Twiddles<P, E, T> tw;
    tw.load(t, twN, 2 * Q);
    fft_inv<P, E, Q * C, T>(v, t, lds, tw);
    const T up = scale_finish<T>(gscale, unit);
    if (up != T(1))
#pragma unroll
        for (int a = 0; a < Q * C; ++a)
#pragma unroll
            for (int e = 0; e < E; ++e) v[a][e] = scale(v[a][e], up);
    // z[Qn + r] back in order through LDS (the transforms' last reads are
    // behind their final barrier), so that each store writes consecutive
    // points
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int r = 0; r < Q; ++r) mir.st(Q * (t + e * TH) + r, v[Q * c + r][e]);
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const Lds<T> mir = rowq_mirror_lds<T, P, Q>(buf, gi, G, c);
            cx<T> *yz = reinterpret_cast<cx<T> *>((c == 0 ? out0 : out1) + (size_t)i * N);
#pragma unroll
            for (int u = 0; u < Q * E; ++u) store_stream(&yz[t + u * TH], mir.ld(t + u * TH));
        }
    }
}

}  // namespace pf
