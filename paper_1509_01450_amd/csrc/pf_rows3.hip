// pf_rows3.hip -- the row transforms along phi for N_phi = 6 P (P a power of
// two): pass A and pass C of grids whose azimuthal count is three times a
// power of two.  Power-of-two rows take the kernels of pf_passes.hip.
//
// A real row of N = 2 M points, M = 3 P, goes through the M-point complex
// transform of z[m] = x[2m] + i x[2m+1], as in the power-of-two rows; that
// transform is split by decimation in time into three P-point transforms
// Y_r of z[3n + r] (r = 0, 1, 2), run by the power-of-two stages of
// fft_core.hpp as six (or three) transforms held together, and one radix-3
// step in registers:
//   Z[k + jP] = sum_r (W_M^(r k) Y_r[k]) W_3^(r j),   k in [0, P), j = 0, 1, 2,
// W_M = exp(-2 pi i / M), W_3 = exp(-2 pi i / 3).  Thread t holds the points
// k = t + e TH (TH = P / E) of all three Y_r, so it forms Z at k, k + P and
// k + 2P itself.  The packed half spectrum (bin 0 = (X_0, X_M)) then follows
// from Z and its mirror bins M - k as in the power-of-two rows.  The
// inverse (pass C) runs the same steps backwards:
//   z[3n + r] = sum_k' W_P^(-n k') [W_M^(-r k') sum_j Z[k' + jP] W_3^(-r j)].
// Workgroup: G rows x TH threads; LDS: C G row3_len(P) complex, per channel
// and row the three P-point regions, reused for the mirror exchange.
#include "pass_bodies.hpp"
#include "pf_common.hpp"

namespace pf {

namespace {

// LDS slots per row and channel: three padded P-point regions, or one padded
// 3P-point region for the mirror exchange, whichever is longer
__host__ __device__ constexpr int row3_len(int P) {
    return 3 * padded_len(P) > padded_len(3 * P) ? 3 * padded_len(P) : padded_len(3 * P);
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

template <typename T, int P, int C>
__device__ __forceinline__ void row3_sub_lds(cx<T> *buf, int gi, int G, Lds<T> (&lds)[3 * C]) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r)
            lds[3 * c + r] = Lds<T>{buf, (c * G + gi) * row3_len(P) + r * padded_len(P), 1};
}

template <typename T, int P>
__device__ __forceinline__ Lds<T> row3_mirror_lds(cx<T> *buf, int gi, int G, int c) {
    return Lds<T>{buf, (c * G + gi) * row3_len(P), 1};
}

// Pass A: rows of in0 (and in1 for C = 2) -> packed half spectra
// (out: [n_rows][M] complex for C = 1, pairs for C = 2).
template <typename T, int P, int E, int C>
__device__ __forceinline__ void body_rows_r2c3(int unit, int G, cx<T> *__restrict__ buf,
                                               const T *__restrict__ in0,
                                               const T *__restrict__ in1, int n_rows,
                                               cx<T> *__restrict__ out,
                                               const cx<T> *__restrict__ twN,
                                               unsigned *__restrict__ gscale) {
    constexpr int TH = P / E;
    constexpr int M = 3 * P;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0
    Lds<T> lds[3 * C];
    row3_sub_lds<T, P, C>(buf, gi, G, lds);

    // z[3n + r] for n = t + e TH: three neighbouring complex values
    cx<T> v[3 * C][E];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<T> *xz = reinterpret_cast<const cx<T> *>((c == 0 ? in0 : in1) + (size_t)i * N);
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int r = 0; r < 3; ++r) v[3 * c + r][e] = xz[3 * (t + e * TH) + r];
    }
    Twiddles<P, E, T> tw;
    tw.load(t, twN, 6);   // the P-point table inside the N-point one
#pragma unroll
    for (int a = 0; a < 3 * C; ++a)
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!active) v[a][e] = cx<T>{T(0), T(0)};
    scale_note<T, E, 3 * C>(gscale, v);
    fft_fwd<P, E, 3 * C, T>(v, t, lds, tw);

    // the radix-3 step: Z at k, k + P, k + 2P, in place of Y_0, Y_1, Y_2
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * TH;
        const cx<T> w1 = twN[2 * k], w2 = twN[4 * k];   // W_M^k, W_M^(2k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            cx<T> z0, z1, z2;
            dft3<T, false>(v[3 * c][e], cmul(v[3 * c + 1][e], w1), cmul(v[3 * c + 2][e], w2), z0,
                           z1, z2);
            v[3 * c][e] = z0;
            v[3 * c + 1][e] = z1;
            v[3 * c + 2][e] = z2;
        }
    }
    // mirror bins through LDS (the transforms' last reads are behind their
    // final barrier; a one-stage transform read nothing)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = row3_mirror_lds<T, P>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) mir.st(t + e * TH + j * P, v[3 * c + j][e]);
    }
    __syncthreads();
    // the packed half spectrum, in place
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = row3_mirror_lds<T, P>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                const cx<T> zk = v[3 * c + j][e], zm = mir.ld(k == 0 ? 0 : M - k);
                const cx<T> ev = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
                // (zk - conj zm) / (2i)
                const cx<T> od = {T(0.5) * (zk.y + zm.y), -T(0.5) * (zk.x - zm.x)};
                cx<T> x = cmac(ev, twN[k], od);
                if (k == 0) x = cx<T>{zk.x + zk.y, zk.x - zk.y};   // (X_0, X_M), both real
                v[3 * c + j][e] = x;
            }
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                if constexpr (C == 1) {
                    store_stream(&out[(size_t)i * M + k], v[j][e]);
                } else {
                    cx2<T> *orow = reinterpret_cast<cx2<T> *>(out) + (size_t)i * M;
                    store_stream(&orow[k], cx2<T>{v[j][e], v[3 + j][e]});
                }
            }
    }
}

// Pass C: packed half rows -> real rows of out0 (and out1), unnormalised
// inverse; turn in [0, N) turns the rows by that many points (bin k times
// exp(-2 pi i k turn / N)), as the power-of-two rows.
template <typename T, int P, int E, int C>
__device__ __forceinline__ void body_rows_c2r3(int unit, int G, cx<T> *__restrict__ buf,
                                               const cx<T> *__restrict__ in, int n_rows,
                                               T *__restrict__ out0, T *__restrict__ out1,
                                               const cx<T> *__restrict__ twN,
                                               unsigned *__restrict__ gscale, int turn) {
    constexpr int TH = P / E;
    constexpr int M = 3 * P;
    constexpr int N = 2 * M;
    const int gi = threadIdx.x / TH, t = threadIdx.x % TH;
    const int row = unit * G + gi;
    const bool active = row < n_rows;
    const int i = active ? row : 0;   // inactive lanes read row 0

    // bins k = t + e TH + j P of channel c at v[3c + j][e]
    cx<T> v[3 * C][E];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH + j * P;
            if constexpr (C == 1) {
                v[j][e] = in[(size_t)i * M + k];
            } else {
                const cx2<T> a = reinterpret_cast<const cx2<T> *>(in)[(size_t)i * M + k];
                v[j][e] = a.a;
                v[3 + j][e] = a.b;
            }
        }
    if (turn) {   // uniform
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                const cx<T> ph = twN[(k * turn) % N];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    cx<T> &x = v[3 * c + j][e];
                    if (k == 0)   // packed (X_0, X_M): X_M times (-1)^turn
                        x.y = (turn & 1) ? -x.y : x.y;
                    else
                        x = cmul(x, ph);
                }
            }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = row3_mirror_lds<T, P>(buf, gi, G, c);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) mir.st(t + e * TH + j * P, v[3 * c + j][e]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const Lds<T> mir = row3_mirror_lds<T, P>(buf, gi, G, c);
        // Z[k] of the complex transform, in place
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * TH + j * P;
                cx<T> a = v[3 * c + j][e], m = mir.ld(k == 0 ? 0 : M - k);
                if (k == 0) {   // unpack bin 0 = (X_0, X_M)
                    m = cx<T>{a.y, T(0)};
                    a = cx<T>{a.x, T(0)};
                }
                const cx<T> s = {a.x + m.x, a.y - m.y};   // X[k] + conj X[M-k]
                const cx<T> d = {a.x - m.x, a.y + m.y};   // X[k] - conj X[M-k]
                const cx<T> w = twN[k];
                const cx<T> iw = {w.y, w.x};   // s + i d exp(+2 pi i k / N)
                v[3 * c + j][e] = cmac(s, d, iw);
            }
        // the inverse radix-3 step: U_r[k'] = W_M^(-r k') sum_j Z[k' + jP] W_3^(-r j),
        // in place of Z at k' + rP
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * TH;
            const cx<T> w1 = twN[2 * k], w2 = twN[4 * k];
            cx<T> b0, b1, b2;
            dft3<T, true>(v[3 * c][e], v[3 * c + 1][e], v[3 * c + 2][e], b0, b1, b2);
            v[3 * c][e] = b0;
            v[3 * c + 1][e] = cmulc(b1, w1);
            v[3 * c + 2][e] = cmulc(b2, w2);
        }
    }
    __syncthreads();   // mirror reads done before the transforms reuse buf
    Lds<T> lds[3 * C];
    row3_sub_lds<T, P, C>(buf, gi, G, lds);
    Twiddles<P, E, T> tw;
    tw.load(t, twN, 6);
    fft_inv<P, E, 3 * C, T>(v, t, lds, tw);
    const T up = scale_finish<T>(gscale, unit);
    if (up != T(1))
#pragma unroll
        for (int a = 0; a < 3 * C; ++a)
#pragma unroll
            for (int e = 0; e < E; ++e) v[a][e] = scale(v[a][e], up);
    if (active) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            cx<T> *yz = reinterpret_cast<cx<T> *>((c == 0 ? out0 : out1) + (size_t)i * N);
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int r = 0; r < 3; ++r) store_stream(&yz[3 * (t + e * TH) + r], v[3 * c + r][e]);
        }
    }
}

template <typename T, int P, int E, int C>
__global__ __launch_bounds__(512) void k_rows_r2c3(const T *__restrict__ in0,
                                                   const T *__restrict__ in1, int n_rows,
                                                   cx<T> *__restrict__ out,
                                                   const cx<T> *__restrict__ twN,
                                                   unsigned *__restrict__ gscale) {
    extern __shared__ unsigned char smem_raw[];
    body_rows_r2c3<T, P, E, C>(blockIdx.x, blockDim.x / (P / E),
                               reinterpret_cast<cx<T> *>(smem_raw), in0, in1, n_rows, out, twN,
                               gscale);
}

template <typename T, int P, int E, int C>
__global__ __launch_bounds__(512) void k_rows_c2r3(const cx<T> *__restrict__ in, int n_rows,
                                                   T *__restrict__ out0, T *__restrict__ out1,
                                                   const cx<T> *__restrict__ twN,
                                                   unsigned *__restrict__ gscale, int turn) {
    extern __shared__ unsigned char smem_raw[];
    body_rows_c2r3<T, P, E, C>(blockIdx.x, blockDim.x / (P / E),
                               reinterpret_cast<cx<T> *>(smem_raw), in, n_rows, out0, out1, twN,
                               gscale, turn);
}

template <typename K>
int allow_lds3(K kern, size_t lds) {
    if (lds > 64 * 1024)
        PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PF_OK;
}

template <typename T>
struct Disp3 {
    template <int P, int E, int C>
    static int r2c(const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g) {
        if constexpr (E <= P) {
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * row3_len(P) * sizeof(cx<T>);
            int rc = allow_lds3(k_rows_r2c3<T, P, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_r2c3<T, P, E, C>), dim3(blocks), dim3(G * (P / E)), lds, st,
                               in0, in1, n_rows, out, tw, g);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of 3 x %d points cannot take %d points per thread", P, E);
        return PF_EUNSUPPORTED;
    }
    template <int P, int E, int C>
    static int c2r(const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g, int turn) {
        if constexpr (E <= P) {
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * row3_len(P) * sizeof(cx<T>);
            int rc = allow_lds3(k_rows_c2r3<T, P, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_c2r3<T, P, E, C>), dim3(blocks), dim3(G * (P / E)), lds, st,
                               in, n_rows, o0, o1, tw, g, turn);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of 3 x %d points cannot take %d points per thread", P, E);
        return PF_EUNSUPPORTED;
    }
    template <int P>
    static int r2c_e(int E, const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw,
                     int G, hipStream_t st, unsigned *g) {
        if (in1) {
            if (E == 4) return r2c<P, 4, 2>(in0, in1, n_rows, out, tw, G, st, g);
            if (E == 8) return r2c<P, 8, 2>(in0, in1, n_rows, out, tw, G, st, g);
        } else {
            if (E == 4) return r2c<P, 4, 1>(in0, in1, n_rows, out, tw, G, st, g);
            if (E == 8) return r2c<P, 8, 1>(in0, in1, n_rows, out, tw, G, st, g);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int P>
    static int c2r_e(int E, const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                     hipStream_t st, unsigned *g, int turn) {
        if (o1) {
            if (E == 4) return c2r<P, 4, 2>(in, n_rows, o0, o1, tw, G, st, g, turn);
            if (E == 8) return c2r<P, 8, 2>(in, n_rows, o0, o1, tw, G, st, g, turn);
        } else {
            if (E == 4) return c2r<P, 4, 1>(in, n_rows, o0, o1, tw, G, st, g, turn);
            if (E == 8) return c2r<P, 8, 1>(in, n_rows, o0, o1, tw, G, st, g, turn);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
};

#define PF_SWITCH_P3(v, F, ...)                            \
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
        default:                                           \
            set_error("no row transform of 3 x %d points", v); \
            return PF_EUNSUPPORTED;                        \
    }

}  // namespace

size_t rows3_lds_bytes(int P, int G, int C, bool f64) {
    return (size_t)C * G * row3_len(P) * (f64 ? 16 : 8);
}

template <typename T>
int launch_rows_r2c3(int M, const T *in0, const T *in1, int n_rows, cx<T> *out,
                     const cx<T> *twN, Shape s, hipStream_t st, unsigned *g) {
    PF_SWITCH_P3(M / 3, Disp3<T>::template r2c_e, s.E, in0, in1, n_rows, out, twN, s.G, st, g);
}

template <typename T>
int launch_rows_c2r3(int M, const cx<T> *in, int n_rows, T *out0, T *out1, const cx<T> *twN,
                     Shape s, hipStream_t st, unsigned *g, int turn) {
    PF_SWITCH_P3(M / 3, Disp3<T>::template c2r_e, s.E, in, n_rows, out0, out1, twN, s.G, st, g,
                 turn);
}

template int launch_rows_r2c3<float>(int, const float *, const float *, int, cx<float> *,
                                     const cx<float> *, Shape, hipStream_t, unsigned *);
template int launch_rows_r2c3<double>(int, const double *, const double *, int, cx<double> *,
                                      const cx<double> *, Shape, hipStream_t, unsigned *);
template int launch_rows_c2r3<float>(int, const cx<float> *, int, float *, float *,
                                     const cx<float> *, Shape, hipStream_t, unsigned *, int);
template int launch_rows_c2r3<double>(int, const cx<double> *, int, double *, double *,
                                      const cx<double> *, Shape, hipStream_t, unsigned *, int);

}  // namespace pf
