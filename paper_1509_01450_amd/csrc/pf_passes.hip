// pf_passes.hip -- the per-call hot path: standalone kernels of the row
// transforms along phi and of the fused column pass along u = ln r, forward
// and transpose, and their runtime dispatch.  The pass bodies (and the
// description of the data flow) are in pass_bodies.hpp.
#include "pass_bodies.hpp"
#include "pf_common.hpp"

namespace pf {

// Standalone kernels: one unit per workgroup.  Column groups are remapped
// so the groups an XCD runs are contiguous: workgroups are dispatched
// round-robin over the 8 XCDs (block b runs on XCD b % 8), and neighbouring
// columns share cache lines of the row-major intermediates.
__device__ __forceinline__ int xcd_group(int b, int per_xcd) { return (b & 7) * per_xcd + (b >> 3); }

// The one-channel row kernels take one extra row of its own buffers (xin ->
// xout, the origin wedges' row) in one more workgroup (n_x = 1), the first
// of the grid so that it does not trail the others, and so that it costs no
// launch of its own.
template <typename T, int M, int E, int C>
__global__ __launch_bounds__(512) void k_rows_r2c(const T *__restrict__ in0,
                                                  const T *__restrict__ in1, int n_rows,
                                                  cx<T> *__restrict__ out,
                                                  const cx<T> *__restrict__ twN,
                                                  unsigned *__restrict__ gscale,
                                                  const T *__restrict__ xin,
                                                  cx<T> *__restrict__ xout, int n_x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = blockDim.x / (M / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        if (n_x && blockIdx.x == 0) {   // workgroup-uniform
            body_rows_r2c<T, M, E, 1>(0, G, buf, xin, nullptr, 1, xout, twN, gscale);
            return;
        }
    body_rows_r2c<T, M, E, C>(blockIdx.x - n_x, G, buf, in0, in1, n_rows, out, twN, gscale);
}

template <typename T, int M, int E, int C>
__global__ __launch_bounds__(512) void k_rows_c2r(const cx<T> *__restrict__ in, int n_rows,
                                                  T *__restrict__ out0, T *__restrict__ out1,
                                                  const cx<T> *__restrict__ twN,
                                                  unsigned *__restrict__ gscale, int turn,
                                                  const cx<T> *__restrict__ xin,
                                                  T *__restrict__ xout, int n_x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = blockDim.x / (M / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        if (n_x && blockIdx.x == 0) {   // workgroup-uniform
            body_rows_c2r<T, M, E, 1>(0, G, buf, xin, 1, xout, nullptr, twN, gscale, turn);
            return;
        }
    body_rows_c2r<T, M, E, C>(blockIdx.x - n_x, G, buf, in, n_rows, out0, out1, twN, gscale,
                              turn);
}

// Forward column pass for any G, with one dynamic LDS array: used where the
// static-LDS kernel below has no instance (columns of fewer than 64
// threads, more than four columns per workgroup, or static LDS beyond
// 144 KB).  In FP32 it prefetches the radial pairs into the same array, so
// the compiler waits for them before the first exchange.
// SO: slope order (4: five-point slopes, c4 their coefficient; only this
// kernel and k_cols_adj have instances of it).
template <typename T, int L, int E, int SO = 2>
__global__ __launch_bounds__(512) void k_cols_fwd(const cx<T> *__restrict__ S,
                                                  cx2<T> *__restrict__ Z,
                                                  const cx2<T> *__restrict__ spec, int H, int n_r,
                                                  int n_out, int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL, int per_xcd,
                                                  int n_groups, unsigned *__restrict__ gscale,
                                                  T c4) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;  // whole workgroup leaves together
    const int G = blockDim.x / (L / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    body_cols_fwd<T, L, E, sizeof(T) == 4, SO>(
        grp, G, buf, S, Z, spec, H, n_r, n_out, ldspec, ca, c0, cn, twL,
        reinterpret_cast<cx2<T> *>(buf + (size_t)G * padded_len(L)), gscale, c4);
}

// Forward column pass with G fixed at compile time: the transform buffer
// and the radial spectrum prefetch region are two static LDS arrays,
// so the prefetch stays in flight while the column is transformed (the
// compiler sees that the transform's LDS accesses cannot touch the
// prefetch region; with one dynamic LDS array it waits for the prefetch
// before the first exchange).
template <typename T, int L, int E, int G, int SO = 2>
__global__ __launch_bounds__(512) void k_cols_fwd_pf(const cx<T> *__restrict__ S,
                                                     cx2<T> *__restrict__ Z,
                                                     const cx2<T> *__restrict__ spec, int H,
                                                     int n_r, int n_out, int ldspec, T ca, T c0,
                                                     T cn, const cx<T> *__restrict__ twL,
                                                     int per_xcd, int n_groups,
                                                     unsigned *__restrict__ gscale, T c4) {
    __shared__ cx<T> fbuf[G * padded_len(L)];
    __shared__ cx2<T> spl[G * spec_prefetch_len<L, E>()];
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;  // whole workgroup leaves together
    body_cols_fwd<T, L, E, true, SO>(grp, G, fbuf, S, Z, spec, H, n_r, n_out, ldspec, ca, c0,
                                     cn, twL, spl, gscale, c4);
}

// n_r: rows of D (source rows), n_v: rows of V (destination rows).
template <typename T, int L, int E, int SO = 2>
__global__ __launch_bounds__(512) void k_cols_adj(const cx2<T> *__restrict__ V,
                                                  cx<T> *__restrict__ D,
                                                  const cx2<T> *__restrict__ spec, int H, int n_r,
                                                  int ldspec, T ca, T c0, T cn,
                                                  const cx<T> *__restrict__ twL, int per_xcd,
                                                  int n_groups, unsigned *__restrict__ gscale,
                                                  T c4, int n_v) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;
    body_cols_adj<T, L, E, false, SO>(grp, blockDim.x / (L / E),
                                      reinterpret_cast<cx<T> *>(smem_raw), V, D, spec, H, n_r,
                                      ldspec, ca, c0, cn, twL, nullptr, gscale, c4, n_v);
}

// Transpose column pass with G fixed at compile time and the radial
// spectrum prefetch in a static LDS array of its own (as k_cols_fwd_pf).
template <typename T, int L, int E, int G, int SO = 2>
__global__ __launch_bounds__(512) void k_cols_adj_pf(const cx2<T> *__restrict__ V,
                                                     cx<T> *__restrict__ D,
                                                     const cx2<T> *__restrict__ spec, int H,
                                                     int n_r, int ldspec, T ca, T c0, T cn,
                                                     const cx<T> *__restrict__ twL, int per_xcd,
                                                     int n_groups,
                                                     unsigned *__restrict__ gscale, T c4,
                                                     int n_v) {
    __shared__ cx<T> fbuf[G * padded_len(L)];
    __shared__ cx2<T> spl[G * spec_prefetch_len<L, E>()];
    const int grp = xcd_group(blockIdx.x, per_xcd);
    if (grp >= n_groups) return;  // whole workgroup leaves together
    body_cols_adj<T, L, E, true, SO>(grp, G, fbuf, V, D, spec, H, n_r, ldspec, ca, c0, cn, twL,
                                     spl, gscale, c4, n_v);
}

// ---------------------------------------------------------------------------
// Runtime dispatch onto the template instantiations.
// ---------------------------------------------------------------------------
// Row shapes are checked for the two-channel passes (the larger LDS need):
// 2 G padded_len(M) complex within 144 KB.
bool valid_shape_rows(int M, Shape s, bool f64) {
    const int Q = row_factor(M);
    if (Q == 0) return false;
    if (Q > 1) {   // M = Q P: Q P-point transforms per channel
        const int P = M / Q;
        if (P < 4 || P > (Q == 3 ? 1024 : 256)) return false;
        // points per thread: 4, or 8 in FP32 (Q = 3); 2 (Q = 9): more spill
        if (Q == 3 ? !(s.E == 4 || (s.E == 8 && !f64)) : s.E != 2) return false;
        if (s.E > P) return false;
        if (s.G < 1 || (P / s.E) * s.G > 512) return false;
        return rowsq_lds_bytes(P, Q, s.G, 2, f64) <= 144 * 1024;
    }
    if (!(s.E == 4 || s.E == 8 || s.E == 16) || s.E > M) return false;
    const int th = M / s.E;
    if (s.G < 1 || th * s.G > 512) return false;
    const size_t lds = (size_t)2 * s.G * padded_len(M) * (f64 ? 16 : 8);
    return lds <= 144 * 1024;
}

// Column pass LDS: G padded_len(L) complex for the transforms and, when
// the radial spectra are prefetched, G spec_prefetch_len<L, E> pairs
// (L/2 + 1 rounded up to a multiple of max(64, L/E)).
size_t cols_lds_bytes(int L, int E, int G, bool f64, bool prefetch) {
    const size_t fft = (size_t)G * padded_len(L) * (f64 ? 16 : 8);
    const int q = L / E > 64 ? L / E : 64;
    const size_t pf = prefetch ? (size_t)G * (((L / 2 + 1) + q - 1) / q * q) * (f64 ? 32 : 16) : 0;
    return fft + pf;
}

bool valid_shape_cols(int L, Shape s, bool f64) {
    if (!(s.E == 8 || s.E == 16) || s.E > L) return false;
    const int th = L / s.E;
    if (s.G < 1 || th * s.G > 512) return false;
    // G a power of two: the column sums of the transpose combine the lanes
    // of a column by exchanges at lane distances G, 2G, ... (interleaved
    // columns); whole waves: the prefetch and the column sums count waves
    if ((s.G & (s.G - 1)) != 0 || (th * s.G) % 64 != 0) return false;
    // FP32 shapes keep room for the prefetch (every FP32 forward kernel
    // takes it); FP64 falls back to the kernel without it when the static
    // prefetch kernel does not fit
    return cols_lds_bytes(L, s.E, s.G, f64, !f64) <= 144 * 1024;
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

// The static-LDS column kernel for a compile-time G, when its LDS
// (transform buffer and prefetch region) fits the 144 KB the shape check
// allows, or 159 KB for a workgroup of 512 threads (one per CU whatever its
// LDS: the registers of a column body allow no more); false (nothing
// launched) otherwise.
template <typename T, int N, int E, int G>
constexpr bool cols_pf_fits() {
    return G * (N / E) <= 512 &&
           (size_t)G * padded_len(N) * sizeof(cx<T>) +
                   (size_t)G * spec_prefetch_len<N, E>() * sizeof(cx2<T>) <=
               (size_t)(G * (N / E) == 512 ? 159 : 144) * 1024;
}

// Slope order 4 has static-LDS instances for the points per thread its
// precision tunes to (FP32 E = 16, FP64 E = 8) only; other shapes take the
// dynamic-LDS kernels.
template <typename T, int E, int SO>
constexpr bool so_pf_instance() {
    return SO == 2 || (sizeof(T) == 4 ? E == 16 : E == 8);
}

template <typename T, int N, int E, int G, int SO>
bool launch_cols_pf(dim3 grid, hipStream_t st, const cx<T> *S, cx2<T> *Z, const cx2<T> *spec,
                    const Plan &p, T ca, T c0, T cn, T c4, const cx<T> *tw, int per_xcd,
                    int n_groups, unsigned *g) {
    if constexpr (cols_pf_fits<T, N, E, G>() && so_pf_instance<T, E, SO>()) {
        hipLaunchKernelGGL((k_cols_fwd_pf<T, N, E, G, SO>), grid, dim3(G * (N / E)), 0, st, S,
                           Z, spec, p.H, p.n_in, p.n_r, p.ldspec, ca, c0, cn, tw, per_xcd,
                           n_groups, g, c4);
        return true;
    }
    return false;
}

template <typename T, int N, int E, int G, int SO>
bool launch_cols_adj_pf(dim3 grid, hipStream_t st, const cx2<T> *V, cx<T> *D,
                        const cx2<T> *spec, const Plan &p, T ca, T c0, T cn, T c4,
                        const cx<T> *tw, int per_xcd, int n_groups, unsigned *g) {
    if constexpr (cols_pf_fits<T, N, E, G>() && so_pf_instance<T, E, SO>()) {
        hipLaunchKernelGGL((k_cols_adj_pf<T, N, E, G, SO>), grid, dim3(G * (N / E)), 0, st, V,
                           D, spec, p.H, p.n_in, p.ldspec, ca, c0, cn, tw, per_xcd, n_groups, g,
                           c4, p.n_r);
        return true;
    }
    return false;
}

template <typename T>
struct Disp {
    template <int N, int E, int C>
    static int r2c(const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g, const T *xin, cx<T> *xout) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * padded_len(N) * sizeof(cx<T>);
            int rc = allow_lds(k_rows_r2c<T, N, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_r2c<T, N, E, C>), dim3(blocks + (xin ? 1 : 0)),
                               dim3(G * TH), lds, st, in0, in1, n_rows, out, tw, g, xin, xout,
                               xin ? 1 : 0);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N, int E, int C>
    static int c2r(const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                   hipStream_t st, unsigned *g, int turn, const cx<T> *xin, T *xout) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int blocks = (n_rows + G - 1) / G;
            const size_t lds = (size_t)C * G * padded_len(N) * sizeof(cx<T>);
            int rc = allow_lds(k_rows_c2r<T, N, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_rows_c2r<T, N, E, C>), dim3(blocks + (xin ? 1 : 0)),
                               dim3(G * TH), lds, st, in, n_rows, o0, o1, tw, g, turn, xin,
                               xout, xin ? 1 : 0);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N, int E, bool ADJ>
    static int cols(const Plan &p, const cx<T> *a, cx<T> *o, const cx<T> *spec, const cx<T> *tw,
                    int G, hipStream_t st, unsigned *g) {
        return p.so == 4 ? cols_so<N, E, ADJ, 4>(p, a, o, spec, tw, G, st, g)
                         : cols_so<N, E, ADJ, 2>(p, a, o, spec, tw, G, st, g);
    }
    template <int N, int E, bool ADJ, int SO>
    static int cols_so(const Plan &p, const cx<T> *a, cx<T> *o, const cx<T> *spec,
                       const cx<T> *tw, int G, hipStream_t st, unsigned *g) {
        if constexpr (E <= N) {
            constexpr int TH = N / E;
            const int n_groups = (p.H + G - 1) / G;
            const int per_xcd = (n_groups + 7) / 8;
            const int blocks = per_xcd * 8;
            // dynamic-LDS kernels: only the FP32 forward one prefetches
            const size_t lds = cols_lds_bytes(N, E, G, sizeof(T) == 8, !ADJ && sizeof(T) == 4);
            const T ca = T(p.ca), c0 = T(p.c0), cn = T(p.cn), c4 = T(p.c4);
            const cx2<T> *sp = reinterpret_cast<const cx2<T> *>(spec);
            if constexpr (TH >= 64) {
                // the prefetch's 32-bit offsets cover a spectrum half
                if ((size_t)p.H * p.ldspec * sizeof(cx2<T>) >= ((size_t)1 << 31)) {
                    set_error("spectra too large for the column pass prefetch");
                    return PF_EUNSUPPORTED;
                }
                const dim3 grid(blocks);
                bool done;
                if (ADJ) {
                    const cx2<T> *v = reinterpret_cast<const cx2<T> *>(a);
                    done = G == 1   ? launch_cols_adj_pf<T, N, E, 1, SO>(grid, st, v, o, sp, p, ca,
                                                                         c0, cn, c4, tw, per_xcd,
                                                                         n_groups, g)
                           : G == 2 ? launch_cols_adj_pf<T, N, E, 2, SO>(grid, st, v, o, sp, p, ca,
                                                                         c0, cn, c4, tw, per_xcd,
                                                                         n_groups, g)
                           : G == 4 ? launch_cols_adj_pf<T, N, E, 4, SO>(grid, st, v, o, sp, p, ca,
                                                                         c0, cn, c4, tw, per_xcd,
                                                                         n_groups, g)
                                    : false;
                } else {
                    cx2<T> *z = reinterpret_cast<cx2<T> *>(o);
                    done = G == 1   ? launch_cols_pf<T, N, E, 1, SO>(grid, st, a, z, sp, p, ca, c0,
                                                                     cn, c4, tw, per_xcd, n_groups,
                                                                     g)
                           : G == 2 ? launch_cols_pf<T, N, E, 2, SO>(grid, st, a, z, sp, p, ca, c0,
                                                                     cn, c4, tw, per_xcd, n_groups,
                                                                     g)
                           : G == 4 ? launch_cols_pf<T, N, E, 4, SO>(grid, st, a, z, sp, p, ca, c0,
                                                                     cn, c4, tw, per_xcd, n_groups,
                                                                     g)
                                    : false;
                }
                if (done) {
                    PF_HIP(hipGetLastError());
                    return PF_OK;
                }
            }
            if (ADJ) {
                int rc = allow_lds(k_cols_adj<T, N, E, SO>, lds);
                if (rc) return rc;
                hipLaunchKernelGGL((k_cols_adj<T, N, E, SO>), dim3(blocks), dim3(G * TH), lds, st,
                                   reinterpret_cast<const cx2<T> *>(a), o, sp, p.H, p.n_in,
                                   p.ldspec, ca, c0, cn, tw, per_xcd, n_groups, g, c4, p.n_r);
            } else {
                int rc = allow_lds(k_cols_fwd<T, N, E, SO>, lds);
                if (rc) return rc;
                hipLaunchKernelGGL((k_cols_fwd<T, N, E, SO>), dim3(blocks), dim3(G * TH), lds, st,
                                   a, reinterpret_cast<cx2<T> *>(o), sp, p.H, p.n_in, p.n_r,
                                   p.ldspec, ca, c0, cn, tw, per_xcd, n_groups, g, c4);
            }
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("column transform of %d points cannot take %d points per thread", N, E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int r2c_e(int E, const T *in0, const T *in1, int n_rows, cx<T> *out, const cx<T> *tw,
                     int G, hipStream_t st, unsigned *g, const T *xin, cx<T> *xout) {
        if (in1) {
            switch (E) {
                case 4: return r2c<N, 4, 2>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
                case 8: return r2c<N, 8, 2>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
                case 16: return r2c<N, 16, 2>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
            }
        } else {
            switch (E) {
                case 4: return r2c<N, 4, 1>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
                case 8: return r2c<N, 8, 1>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
                case 16: return r2c<N, 16, 1>(in0, in1, n_rows, out, tw, G, st, g, xin, xout);
            }
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int c2r_e(int E, const cx<T> *in, int n_rows, T *o0, T *o1, const cx<T> *tw, int G,
                     hipStream_t st, unsigned *g, int turn, const cx<T> *xin,
                     T *xout) {
        if (o1) {
            switch (E) {
                case 4: return c2r<N, 4, 2>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
                case 8: return c2r<N, 8, 2>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
                case 16: return c2r<N, 16, 2>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
            }
        } else {
            switch (E) {
                case 4: return c2r<N, 4, 1>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
                case 8: return c2r<N, 8, 1>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
                case 16: return c2r<N, 16, 1>(in, n_rows, o0, o1, tw, G, st, g, turn, xin, xout);
            }
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int fwd_e(int E, const Plan &p, const cx<T> *a, cx<T> *o, const cx<T> *spec,
                     const cx<T> *tw, int G, hipStream_t st, unsigned *g) {
        switch (E) {
            case 8: return cols<N, 8, false>(p, a, o, spec, tw, G, st, g);
            case 16: return cols<N, 16, false>(p, a, o, spec, tw, G, st, g);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
    template <int N>
    static int adj_e(int E, const Plan &p, const cx<T> *a, cx<T> *o, const cx<T> *spec,
                     const cx<T> *tw, int G, hipStream_t st, unsigned *g) {
        switch (E) {
            case 8: return cols<N, 8, true>(p, a, o, spec, tw, G, st, g);
            case 16: return cols<N, 16, true>(p, a, o, spec, tw, G, st, g);
        }
        set_error("bad points per thread %d", E);
        return PF_EUNSUPPORTED;
    }
};

}  // namespace

template <typename T>
int launch_rows_r2c(const Plan &p, const T *in0, const T *in1, int n_rows, cx<T> *out,
                    const cx<T> *twN, Shape s, hipStream_t st, unsigned *g, const T *xin,
                    cx<T> *xout) {
    if (xin && in1) {
        set_error("an extra row goes with one-channel row transforms only");
        return PF_EINVAL;
    }
    if (sizeof(T) == 4 && !g) {
        set_error("FP32 passes need the plan's scale words");
        return PF_EINVAL;
    }
    if (!valid_shape_rows(p.M, s, sizeof(T) == 8)) {
        set_error("invalid row shape E=%d G=%d for M=%d", s.E, s.G, p.M);
        return PF_EINVAL;
    }
    if (!is_pow2_int(p.M))
        return launch_rows_r2cq<T>(p.M, in0, in1, n_rows, out, twN, s, st, g, xin, xout);
    PF_SWITCH_POW2(p.M, Disp<T>::template r2c_e, s.E, in0, in1, n_rows, out, twN, s.G, st, g, xin,
                   xout);
}

template <typename T>
int launch_rows_c2r(const Plan &p, const cx<T> *in, int n_rows, T *out0, T *out1,
                    const cx<T> *twN, Shape s, hipStream_t st, unsigned *g, int turn,
                    const cx<T> *xin, T *xout) {
    if (xin && out1) {
        set_error("an extra row goes with one-channel row transforms only");
        return PF_EINVAL;
    }
    if (sizeof(T) == 4 && !g) {
        set_error("FP32 passes need the plan's scale words");
        return PF_EINVAL;
    }
    if (!valid_shape_rows(p.M, s, sizeof(T) == 8)) {
        set_error("invalid row shape E=%d G=%d for M=%d", s.E, s.G, p.M);
        return PF_EINVAL;
    }
    turn %= p.n_phi;
    if (turn < 0) turn += p.n_phi;
    if (!is_pow2_int(p.M))
        return launch_rows_c2rq<T>(p.M, in, n_rows, out0, out1, twN, s, st, g, turn, xin, xout);
    PF_SWITCH_POW2(p.M, Disp<T>::template c2r_e, s.E, in, n_rows, out0, out1, twN, s.G, st, g,
                   turn, xin, xout);
}

template <typename T>
int launch_cols_fwd(const Plan &p, const cx<T> *S, cx<T> *Z, const cx<T> *spec,
                    const cx<T> *twL, Shape s, hipStream_t st, unsigned *g) {
    if (sizeof(T) == 4 && !g) {
        set_error("FP32 passes need the plan's scale words");
        return PF_EINVAL;
    }
    if (!valid_shape_cols(p.L, s, sizeof(T) == 8)) {
        set_error("invalid column shape E=%d G=%d for L=%d", s.E, s.G, p.L);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.L, Disp<T>::template fwd_e, s.E, p, S, Z, spec, twL, s.G, st, g);
}

template <typename T>
int launch_cols_adj(const Plan &p, const cx<T> *V, cx<T> *D, const cx<T> *spec,
                    const cx<T> *twL, Shape s, hipStream_t st, unsigned *g) {
    if (sizeof(T) == 4 && !g) {
        set_error("FP32 passes need the plan's scale words");
        return PF_EINVAL;
    }
    if (!valid_shape_cols(p.L, s, sizeof(T) == 8)) {
        set_error("invalid column shape E=%d G=%d for L=%d", s.E, s.G, p.L);
        return PF_EINVAL;
    }
    PF_SWITCH_POW2(p.L, Disp<T>::template adj_e, s.E, p, V, D, spec, twL, s.G, st, g);
}

#define PF_INSTANTIATE(T)                                                                      \
    template int launch_rows_r2c<T>(const Plan &, const T *, const T *, int, cx<T> *,          \
                                    const cx<T> *, Shape, hipStream_t, unsigned *, const T *,   \
                                    cx<T> *);                                                   \
    template int launch_rows_c2r<T>(const Plan &, const cx<T> *, int, T *, T *, const cx<T> *,  \
                                    Shape, hipStream_t, unsigned *, int, const cx<T> *, T *);   \
    template int launch_cols_fwd<T>(const Plan &, const cx<T> *, cx<T> *, const cx<T> *,        \
                                    const cx<T> *, Shape, hipStream_t, unsigned *);             \
    template int launch_cols_adj<T>(const Plan &, const cx<T> *, cx<T> *, const cx<T> *,        \
                                    const cx<T> *, Shape, hipStream_t, unsigned *);
PF_INSTANTIATE(float)
PF_INSTANTIATE(double)

}  // namespace pf
