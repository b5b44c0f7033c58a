// pf_rows3.hip -- the row transforms along phi for N_phi = 2 Q P with Q = 3
// or 9 and P a power of two: pass A and pass C of grids whose azimuthal
// count is three or nine times a power of two.  Power-of-two rows take the
// kernels of pf_passes.hip.
//
// The bodies (the split into Q power-of-two transforms and the radix-Q step)
// are in rows_q.hpp.
#include "pf_common.hpp"
#include "rows_q.hpp"

namespace pf {

namespace {

// As the power-of-two row kernels: one-channel kernels take one extra row
// of its own buffers (xin -> xout) in one more workgroup (n_x = 1), the
// first of the grid.
template <typename T, int P, int Q, int E, int C>
__global__ __launch_bounds__(512) void k_rows_r2cq(const T *__restrict__ in0,
                                                   const T *__restrict__ in1, int n_rows,
                                                   cx<T> *__restrict__ out,
                                                   const cx<T> *__restrict__ twN,
                                                   unsigned *__restrict__ gscale,
                                                   const T *__restrict__ xin,
                                                   cx<T> *__restrict__ xout, int n_x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = blockDim.x / (P / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        if (n_x && blockIdx.x == 0) {   // workgroup-uniform
            body_rows_r2cq<T, P, Q, E, 1>(0, G, buf, xin, nullptr, 1, xout, twN, gscale);
            return;
        }
    body_rows_r2cq<T, P, Q, E, C>(blockIdx.x - n_x, G, buf, in0, in1, n_rows, out, twN, gscale);
}

template <typename T, int P, int Q, int E, int C>
__global__ __launch_bounds__(512) void k_rows_c2rq(const cx<T> *__restrict__ in, int n_rows,
                                                   T *__restrict__ out0, T *__restrict__ out1,
                                                   const cx<T> *__restrict__ twN,
                                                   unsigned *__restrict__ gscale, int turn,
                                                   const cx<T> *__restrict__ xin,
                                                   T *__restrict__ xout, int n_x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = blockDim.x / (P / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        if (n_x && blockIdx.x == 0) {   // workgroup-uniform
            body_rows_c2rq<T, P, Q, E, 1>(0, G, buf, xin, 1, xout, nullptr, twN, gscale, turn);
            return;
        }
    body_rows_c2rq<T, P, Q, E, C>(blockIdx.x - n_x, G, buf, in, n_rows, out0, out1, twN, gscale,
                                  turn);
}

template <typename K>
int allow_ldsq(K kern, size_t lds) {
    if (lds > 64 * 1024)
        PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PF_OK;
}

template <typename T, int Q>
struct DispQ {
    template <int P, int E, int C>
    static int r2c(const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g, const T *xin, cx<T> *xout) {
        if constexpr (E <= P) {
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * rowq_len(P, Q) * sizeof(cx<T>);
            int rc = allow_ldsq(k_rows_r2cq<T, P, Q, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_r2cq<T, P, Q, E, C>), dim3(blocks + (xin ? 1 : 0)),
                               dim3(G * (P / E)), lds, st, in0, in1, n_rows, out, tw, g, xin,
                               xout, xin ? 1 : 0);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d x %d points cannot take %d points per thread", Q, P, E);
        return PF_EUNSUPPORTED;
    }
    template <int P, int E, int C>
    static int c2r(const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g, int turn, const cx<T> *xin, T *xout) {
        if constexpr (E <= P) {
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * rowq_len(P, Q) * sizeof(cx<T>);
            int rc = allow_ldsq(k_rows_c2rq<T, P, Q, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_c2rq<T, P, Q, E, C>), dim3(blocks + (xin ? 1 : 0)),
                               dim3(G * (P / E)), lds, st, in, n_rows, o0, o1, tw, g, turn, xin,
                               xout, xin ? 1 : 0);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d x %d points cannot take %d points per thread", Q, P, E);
        return PF_EUNSUPPORTED;
    }
    // points per thread: 4 or 8 with Q = 3, 2 with Q = 9
    template <int P>
    static int r2c_e(int E, const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw,
                     int G, hipStream_t st, unsigned *g, const T *xin, cx<T> *xout) {
        constexpr int EA = Q == 3 ? 4 : 2, EB = Q == 3 ? 8 : 2;
        if (in1) {
            if (E == EA) return r2c<P, EA, 2>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
            if (E == EB) return r2c<P, EB, 2>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
        } else {
            if (E == EA) return r2c<P, EA, 1>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
            if (E == EB) return r2c<P, EB, 1>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int P>
    static int c2r_e(int E, const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                     hipStream_t st, unsigned *g, int turn, const cx<T> *xin,
                     T *xout) {
        constexpr int EA = Q == 3 ? 4 : 2, EB = Q == 3 ? 8 : 2;
        if (o1) {
            if (E == EA) return c2r<P, EA, 2>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
            if (E == EB) return c2r<P, EB, 2>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
        } else {
            if (E == EA) return c2r<P, EA, 1>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
            if (E == EB) return c2r<P, EB, 1>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
};

#define PF_SWITCH_P3(v, F, ...)                                \
    switch (v) {                                               \
        case 4: return F<4>(__VA_ARGS__);                      \
        case 8: return F<8>(__VA_ARGS__);                      \
        case 16: return F<16>(__VA_ARGS__);                    \
        case 32: return F<32>(__VA_ARGS__);                    \
        case 64: return F<64>(__VA_ARGS__);                    \
        case 128: return F<128>(__VA_ARGS__);                  \
        case 256: return F<256>(__VA_ARGS__);                  \
        case 512: return F<512>(__VA_ARGS__);                  \
        case 1024: return F<1024>(__VA_ARGS__);                \
        default:                                               \
            set_error("no row transform of 3 x %d points", v); \
            return PF_EUNSUPPORTED;                            \
    }
#define PF_SWITCH_P9(v, F, ...)                                \
    switch (v) {                                               \
        case 4: return F<4>(__VA_ARGS__);                      \
        case 8: return F<8>(__VA_ARGS__);                      \
        case 16: return F<16>(__VA_ARGS__);                    \
        case 32: return F<32>(__VA_ARGS__);                    \
        case 64: return F<64>(__VA_ARGS__);                    \
        case 128: return F<128>(__VA_ARGS__);                  \
        case 256: return F<256>(__VA_ARGS__);                  \
        default:                                               \
            set_error("no row transform of 9 x %d points", v); \
            return PF_EUNSUPPORTED;                            \
    }

}  // namespace

size_t rowsq_lds_bytes(int P, int Q, int G, int C, bool f64) {
    return (size_t)C * G * rowq_len(P, Q) * (f64 ? 16 : 8);
}

template <typename T>
int launch_rows_r2cq(int M, const T *in0, const T *in1, int n_rows, cx<T> *out,
                     const cx<T> *twN, Shape s, hipStream_t st, unsigned *g, const T *xin,
                     cx<T> *xout) {
    using D3 = DispQ<T, 3>;
    using D9 = DispQ<T, 9>;
    if (row_factor(M) == 3)
        PF_SWITCH_P3(M / 3, D3::template r2c_e, s.E, in0, in1, n_rows, out, twN, s.G,
                     st, g, xin, xout);
    if (row_factor(M) == 9)
        PF_SWITCH_P9(M / 9, D9::template r2c_e, s.E, in0, in1, n_rows, out, twN, s.G,
                     st, g, xin, xout);
    set_error("no row transform of %d points", M);
    return PF_EUNSUPPORTED;
}

template <typename T>
int launch_rows_c2rq(int M, const cx<T> *in, int n_rows, T *out0, T *out1, const cx<T> *twN,
                     Shape s, hipStream_t st, unsigned *g, int turn, const cx<T> *xin,
                     T *xout) {
    using D3 = DispQ<T, 3>;
    using D9 = DispQ<T, 9>;
    if (row_factor(M) == 3)
        PF_SWITCH_P3(M / 3, D3::template c2r_e, s.E, in, n_rows, out0, out1, twN, s.G,
                     st, g, turn, xin, xout);
    if (row_factor(M) == 9)
        PF_SWITCH_P9(M / 9, D9::template c2r_e, s.E, in, n_rows, out0, out1, twN, s.G,
                     st, g, turn, xin, xout);
    set_error("no row transform of %d points", M);
    return PF_EUNSUPPORTED;
}

template int launch_rows_r2cq<float>(int, const float *, const float *, int, cx<float> *,
                                     const cx<float> *, Shape, hipStream_t, unsigned *,
                                     const float *, cx<float> *);
template int launch_rows_r2cq<double>(int, const double *, const double *, int, cx<double> *,
                                      const cx<double> *, Shape, hipStream_t, unsigned *,
                                      const double *, cx<double> *);
template int launch_rows_c2rq<float>(int, const cx<float> *, int, float *, float *,
                                     const cx<float> *, Shape, hipStream_t, unsigned *, int,
                                     const cx<float> *, float *);
template int launch_rows_c2rq<double>(int, const cx<double> *, int, double *, double *,
                                      const cx<double> *, Shape, hipStream_t, unsigned *, int,
                                      const cx<double> *, double *);

}  // namespace pf
