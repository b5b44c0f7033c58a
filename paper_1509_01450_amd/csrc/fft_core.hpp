// fft_core.hpp -- workgroup-level complex FFT building blocks for gfx950.
//
// A length-N transform is held by N/E cooperating threads, E points each, in
// registers.  Points are kept in "strided" order: thread t holds element
// t + e * (N/E) in v[e].  The transform runs as Stockham radix-E stages (the
// last one of radix N / E^s when E does not divide evenly), each a set of
// in-register radix-R butterflies; between stages the points go through an
// LDS buffer.  The output comes back in the same strided natural order, so
// a pointwise multiply and the inverse transform can follow in registers
// with no extra exchange.  Twiddles come from a table w[j] = exp(-2 pi i j/N)
// built on the host in extended precision, held per thread in registers.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

namespace pf {

// Words of the FP32 per-grid scale (used by the passes, described in
// pass_bodies.hpp): 64 notes 128 bytes apart, then the word holding the
// exponent; one set of kScaleSet words for the forward map and one for the
// transpose.
constexpr int kScaleWords = 64;
constexpr int kScaleStride = 32;
constexpr int kScaleE = kScaleWords * kScaleStride;
constexpr int kScaleSet = kScaleE + kScaleStride;
constexpr int kScaleFree = 32;   // |e| up to this: no scaling

// complex value, aligned to its full size so that loads, stores and LDS
// accesses are single 64-bit (float) or 128-bit (double) operations
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

// the values of two channels at one point, one aligned 16-byte (FP32) or
// 32-byte (FP64) access
template <typename T>
struct alignas(4 * sizeof(T)) cx2 {
    cx<T> a, b;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }

// Fused multiply-adds written out.  The library is compiled with contraction
// limited to single expressions (-ffp-contract=on), so every rounding step
// is fixed by the source and not by how a kernel happens to be inlined or
// scheduled: the batched kernels, which run the same pass bodies, then give
// the single-disk results bit for bit.  Where a product and a sum are to
// fuse across expressions they go through these.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc + a b
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    return {fmadd(a.x, b.x, fmadd(-a.y, b.y, acc.x)), fmadd(a.x, b.y, fmadd(a.y, b.x, acc.y))};
}
// acc + a conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b) {
    return {fmadd(a.x, b.x, fmadd(a.y, b.y, acc.x)), fmadd(a.y, b.x, fmadd(-a.x, b.y, acc.y))};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }

// ---------------------------------------------------------------------------
// In-register forward DFTs of radix 2, 4, 8, 16 (sign -1).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft2(cx<T> &a, cx<T> &b) {
    cx<T> t = a - b;
    a = a + b;
    b = t;
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T> &a0, cx<T> &a1, cx<T> &a2, cx<T> &a3) {
    cx<T> s0 = a0 + a2, d0 = a0 - a2;
    cx<T> s1 = a1 + a3, d1 = mul_mi(a1 - a3);
    a0 = s0 + s1;
    a2 = s0 - s1;
    a1 = d0 + d1;
    a3 = d0 - d1;
}

template <int R, typename T>
__device__ __forceinline__ void dft(cx<T> *u);

template <>
__device__ __forceinline__ void dft<2, float>(cx<float> *u) { dft2(u[0], u[1]); }
template <>
__device__ __forceinline__ void dft<2, double>(cx<double> *u) { dft2(u[0], u[1]); }
template <>
__device__ __forceinline__ void dft<4, float>(cx<float> *u) { dft4(u[0], u[1], u[2], u[3]); }
template <>
__device__ __forceinline__ void dft<4, double>(cx<double> *u) { dft4(u[0], u[1], u[2], u[3]); }

template <typename T>
__device__ __forceinline__ void dft8_impl(cx<T> *u) {
    const T h = T(0.70710678118654752440084436210484903928);
    // two radix-4 on even / odd, then radix-2 with W8 twiddles
    cx<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    cx<T> o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    // o_k *= exp(-2 pi i k / 8)
    cx<T> w1 = {(o1.x + o1.y) * h, (o1.y - o1.x) * h};   // * (1 - i)/sqrt2
    cx<T> w2 = mul_mi(o2);                               // * -i
    cx<T> w3 = {(o3.y - o3.x) * h, -(o3.x + o3.y) * h};  // * (-1 - i)/sqrt2
    u[0] = e0 + o0;
    u[4] = e0 - o0;
    u[1] = e1 + w1;
    u[5] = e1 - w1;
    u[2] = e2 + w2;
    u[6] = e2 - w2;
    u[3] = e3 + w3;
    u[7] = e3 - w3;
}
template <>
__device__ __forceinline__ void dft<8, float>(cx<float> *u) { dft8_impl(u); }
template <>
__device__ __forceinline__ void dft<8, double>(cx<double> *u) { dft8_impl(u); }

template <typename T>
__device__ __forceinline__ void dft16_impl(cx<T> *u) {
    // 4 x 4 with internal twiddles exp(-2 pi i j k / 16)
    const T c1 = T(0.92387953251128675612818318939678828682);
    const T s1 = T(0.38268343236508977172845998403039886676);
    const T h = T(0.70710678118654752440084436210484903928);
    cx<T> a[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j][0] = u[j];
        a[j][1] = u[j + 4];
        a[j][2] = u[j + 8];
        a[j][3] = u[j + 12];
        dft4(a[j][0], a[j][1], a[j][2], a[j][3]);
    }
    // twiddle a[j][k] by exp(-2 pi i j k / 16)
    const cx<T> w[10] = {{T(1), T(0)}, {c1, -s1}, {h, -h}, {s1, -c1}, {T(0), T(-1)},
                         {-s1, -c1}, {-h, -h}, {-c1, -s1}, {T(-1), T(0)}, {-c1, s1}};
#pragma unroll
    for (int j = 1; j < 4; ++j)
#pragma unroll
        for (int k = 1; k < 4; ++k) a[j][k] = cmul(a[j][k], w[j * k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dft4(a[0][k], a[1][k], a[2][k], a[3][k]);
        u[k] = a[0][k];
        u[k + 4] = a[1][k];
        u[k + 8] = a[2][k];
        u[k + 12] = a[3][k];
    }
}
template <>
__device__ __forceinline__ void dft<16, float>(cx<float> *u) { dft16_impl(u); }
template <>
__device__ __forceinline__ void dft<16, double>(cx<double> *u) { dft16_impl(u); }

// Radix R DFT whose inputs u[R/2 .. R-1] are zero (the first stage of a
// transform of a zero-padded sequence): the first layer of radix-4
// butterflies sees two nonzero inputs each.
template <typename T>
__device__ __forceinline__ void dft4_zh(cx<T> &a0, cx<T> &a1, cx<T> &a2, cx<T> &a3) {
    const cx<T> d1 = mul_mi(a1);
    a2 = a0 - a1;
    a3 = a0 - d1;
    const cx<T> s = a0 + a1;
    a1 = a0 + d1;
    a0 = s;
}

template <int R, typename T>
__device__ __forceinline__ void dft_zh(cx<T> *u) {
    if constexpr (R == 4) {
        dft4_zh(u[0], u[1], u[2], u[3]);
    } else if constexpr (R == 8) {
        const T h = T(0.70710678118654752440084436210484903928);
        cx<T> e0 = u[0], e1 = u[2], e2, e3;
        cx<T> o0 = u[1], o1 = u[3], o2, o3;
        dft4_zh(e0, e1, e2, e3);
        dft4_zh(o0, o1, o2, o3);
        cx<T> w1 = {(o1.x + o1.y) * h, (o1.y - o1.x) * h};
        cx<T> w2 = mul_mi(o2);
        cx<T> w3 = {(o3.y - o3.x) * h, -(o3.x + o3.y) * h};
        u[0] = e0 + o0;
        u[4] = e0 - o0;
        u[1] = e1 + w1;
        u[5] = e1 - w1;
        u[2] = e2 + w2;
        u[6] = e2 - w2;
        u[3] = e3 + w3;
        u[7] = e3 - w3;
    } else {
        static_assert(R == 16, "radix");
        const T c1 = T(0.92387953251128675612818318939678828682);
        const T s1 = T(0.38268343236508977172845998403039886676);
        const T h = T(0.70710678118654752440084436210484903928);
        cx<T> a[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j][0] = u[j];
            a[j][1] = u[j + 4];
            dft4_zh(a[j][0], a[j][1], a[j][2], a[j][3]);
        }
        const cx<T> w[10] = {{T(1), T(0)}, {c1, -s1}, {h, -h}, {s1, -c1}, {T(0), T(-1)},
                             {-s1, -c1}, {-h, -h}, {-c1, -s1}, {T(-1), T(0)}, {-c1, s1}};
#pragma unroll
        for (int j = 1; j < 4; ++j)
#pragma unroll
            for (int k = 1; k < 4; ++k) a[j][k] = cmul(a[j][k], w[j * k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            dft4(a[0][k], a[1][k], a[2][k], a[3][k]);
            u[k] = a[0][k];
            u[k + 4] = a[1][k];
            u[k + 8] = a[2][k];
            u[k + 12] = a[3][k];
        }
    }
}

// x w^k with w = exp(-2 pi i / E), E in {4, 8, 16}, for a k fixed at compile
// time once loops are unrolled: quarter turns are swaps and sign changes,
// the others one complex product by constants.
template <int E, typename T>
__device__ __forceinline__ cx<T> mul_root(cx<T> x, int k) {
    static_assert(E == 4 || E == 8 || E == 16, "roots of unity of order 4, 8 or 16");
    const int q = (((k % E) + E) % E) * (16 / E);   // sixteenths of a turn
    if (q == 0) return x;
    if (q == 4) return {x.y, -x.x};
    if (q == 8) return {-x.x, -x.y};
    if (q == 12) return {-x.y, x.x};
    const T c1 = T(0.92387953251128675612818318939678828682);
    const T s1 = T(0.38268343236508977172845998403039886676);
    const T h = T(0.70710678118654752440084436210484903928);
    // cos and sin of 2 pi q / 16
    const T cs[16] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1, -h, -s1, T(0), s1, h, c1};
    const T c = cs[q], sn = cs[(q + 12) & 15];
    return {x.x * c + x.y * sn, x.y * c - x.x * sn};
}

// acc + x w^k (as mul_root, the product fused into the sum)
template <int E, typename T>
__device__ __forceinline__ cx<T> mul_root_add(cx<T> acc, cx<T> x, int k) {
    static_assert(E == 4 || E == 8 || E == 16, "roots of unity of order 4, 8 or 16");
    const int q = (((k % E) + E) % E) * (16 / E);   // sixteenths of a turn
    if (q == 0) return acc + x;
    if (q == 4) return {acc.x + x.y, acc.y - x.x};
    if (q == 8) return {acc.x - x.x, acc.y - x.y};
    if (q == 12) return {acc.x - x.y, acc.y + x.x};
    const T c1 = T(0.92387953251128675612818318939678828682);
    const T s1 = T(0.38268343236508977172845998403039886676);
    const T h = T(0.70710678118654752440084436210484903928);
    const T cs[16] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1, -h, -s1, T(0), s1, h, c1};
    const T c = cs[q], sn = cs[(q + 12) & 15];
    return {fmadd(x.x, c, fmadd(x.y, sn, acc.x)), fmadd(x.y, c, fmadd(-x.x, sn, acc.y))};
}

// ---------------------------------------------------------------------------
// LDS accessors.  Element i of the FFT group lives at
// base + pad(i) * stride with pad(i) = i + (i >> 4): one unused slot after
// every 16 elements.  The stride-R stores of the early Stockham stages then
// fall on distinct banks (modelled at most 1.33-way for 64 banks of 4 bytes
// and conflict-free for 32, for 8- and 16-byte elements, E = 8 and 16, one
// transform per region or G interleaved columns), and the map splits over
// the sums the stages form: for a power of two P, 0 <= a < P and c a
// multiple of P, pad(a + c) = pad(a) + pad(c) whenever the span of a lies in
// one aligned block of 16 or P is a multiple of 16 -- which holds for the
// exchange reads (t + e TH, t < TH) and for the butterfly writes
// (base + r NS, base = NS R m + k, k < NS).  The per-thread part is formed
// once and every access is that register plus a constant offset.  An
// N-point transform needs padded_len(N) slots.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + n / 16; }

template <typename T>
struct Lds {
    cx<T> *p;
    int base, stride;
    __device__ __forceinline__ int at(int i) const { return base + lds_pad(i) * stride; }
    __device__ __forceinline__ cx<T> ld(int i) const { return p[at(i)]; }
    __device__ __forceinline__ void st(int i, cx<T> v) const { p[at(i)] = v; }
    // element a + c given pa = lds_pad(a) and the split condition above
    __device__ __forceinline__ cx<T> ld_split(int pa, int c) const {
        return p[base + (pa + lds_pad(c)) * stride];
    }
    __device__ __forceinline__ void st_split(int pa, int c, cx<T> v) const {
        p[base + (pa + lds_pad(c)) * stride] = v;
    }
};

// Workgroup barrier for the LDS exchanges: this wave's LDS operations are
// complete (LDS count 0), then the hardware barrier; the memory clobber
// keeps the compiler from moving memory accesses across it.  Unlike
// __syncthreads() it does not wait for the wave's outstanding global memory
// operations, so loads issued before a transform -- including loads into
// another LDS array -- stay in flight across its exchanges.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// Twiddles.  A thread's twiddles depend only on its index t and the stage,
// so they are loaded once from the table into registers (Twiddles::load)
// and reused by every transform the thread runs: no stage waits on a
// global load.  For a stage of radix R and span NS > 1 the thread's
// butterfly q (index b = t + q*TH, k = b mod NS) needs
// w^r = w_{NS R}^{k r} = table[k r N / (NS R)], r = 1..R-1.  Only the
// powers w^1, w^2, w^4, w^8 (log2 R of them) are held; the others are
// formed with at most two complex products (a few ulp), which halves the
// registers the twiddles take.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

template <int N, int E>
__host__ __device__ constexpr int tw_count() {
    int c = 0, ns = 1;
    while (true) {
        const int rem = N / ns;
        const int R = rem >= E ? E : rem;
        const int NB = E / R;
        if (ns > 1) c += NB * ilog2c(R);
        if (ns * R == N) break;
        ns *= R;
    }
    return c;
}

template <int N, int E, typename T>
struct Twiddles {
    static constexpr int COUNT = tw_count<N, E>();
    cx<T> w[COUNT > 0 ? COUNT : 1];

    template <int NS, int OFF>
    __device__ __forceinline__ void load_stage(int t, const cx<T> *__restrict__ tab, int ts) {
        constexpr int TH = N / E;
        constexpr int REM = N / NS;
        constexpr int R = REM >= E ? E : REM;
        constexpr int NB = E / R;
        constexpr int LR = ilog2c(R);
        constexpr bool LAST = (NS * R == N);
        if constexpr (NS > 1) {
            constexpr int STEP = N / (NS * R);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int k = (t + q * TH) & (NS - 1);
#pragma unroll
                for (int j = 0; j < LR; ++j) w[OFF + q * LR + j] = tab[(k * (1 << j) * STEP) * ts];
            }
        }
        if constexpr (!LAST) load_stage<NS * R, OFF + (NS > 1 ? NB * LR : 0)>(t, tab, ts);
    }
    // tab: table exp(-2 pi i j / (N ts)), read with stride ts
    __device__ __forceinline__ void load(int t, const cx<T> *__restrict__ tab, int ts) {
        load_stage<1, 0>(t, tab, ts);
    }
};

// The R-1 twiddles w^1..w^{R-1} of one butterfly from the stored powers
// p[j] = w^(2^j).
template <int R, typename T>
__device__ __forceinline__ void tw_expand(const cx<T> *p, cx<T> *o) {
    o[1] = p[0];
    if constexpr (R > 2) {
        o[2] = p[1];
        o[3] = cmul(p[0], p[1]);
    }
    if constexpr (R > 4) {
        o[4] = p[2];
#pragma unroll
        for (int r = 5; r < 8; ++r) o[r] = cmul(o[r - 4], p[2]);
    }
    if constexpr (R > 8) {
        o[8] = p[3];
#pragma unroll
        for (int r = 9; r < 16; ++r) o[r] = cmul(o[r - 8], p[3]);
    }
}

// ---------------------------------------------------------------------------
// Stockham stages of NV independent transforms held together, each in its
// own LDS region, sharing the stage barriers.  Template parameters: N
// (length), E (points per thread), NS (span of the stage), OFF (offset of the
// stage's twiddles), NV (number of transforms).  All threads of the
// workgroup must call this together (it contains workgroup barriers).
// ---------------------------------------------------------------------------
// F: when not NoScale, an object whose pre() runs after the first stage's
// butterflies, before that stage's barrier, and whose post() runs after the
// barrier; the values read back after the exchange are multiplied by what
// post() returns (a power of two: exact), so a scale found while the first
// stage runs still applies before the later stages.
struct NoScale {};
template <int N, int E, int NS, int OFF, int NV, typename T, bool ZH = false,
          typename F = NoScale>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[NV][E], int t, const Lds<T> (&lds)[NV],
                                           const Twiddles<N, E, T> &tw, F f = F{}) {
    constexpr int TH = N / E;                 // threads per transform
    constexpr int REM = N / NS;
    constexpr int R = REM >= E ? E : REM;     // radix of this stage
    constexpr int NB = E / R;                 // butterflies per thread
    constexpr bool LAST = (NS * R == N);
    static_assert(R >= 2, "radix");
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = t + q * TH;
        const int k = b & (NS - 1);
        cx<T> wr[R];
        if constexpr (NS > 1) tw_expand<R, T>(&tw.w[OFF + q * ilog2c(R)], wr);
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            cx<T> u[R];
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = v[a][q + r * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) u[r] = cmul(u[r], wr[r]);
            }
            if constexpr (ZH && NS == 1 && NB == 1)
                dft_zh<R, T>(u);
            else
                dft<R, T>(u);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[a][q + r * NB] = u[r];
            } else {
                const int pb = lds_pad((b - k) * R + k);
#pragma unroll
                for (int r = 0; r < R; ++r) lds[a].st_split(pb, r * NS, u[r]);
            }
        }
    }
    if constexpr (!LAST) {
        constexpr bool SC = NS == 1 && !std::is_same<F, NoScale>::value;
        T sc = T(1);
        if constexpr (SC) f.pre();
        lds_barrier();
        if constexpr (SC) sc = f.post();
        const int pt = lds_pad(t);
#pragma unroll
        for (int a = 0; a < NV; ++a)
#pragma unroll
            for (int e = 0; e < E; ++e) v[a][e] = lds[a].ld_split(pt, e * TH);
        if constexpr (SC)
            if (sc != T(1))   // uniform: a branch, not a select
#pragma unroll
                for (int a = 0; a < NV; ++a)
#pragma unroll
                    for (int e = 0; e < E; ++e) v[a][e] = scale(v[a][e], sc);
        lds_barrier();
        fft_stages<N, E, NS * R, OFF + (NS > 1 ? NB * ilog2c(R) : 0), NV, T>(v, t, lds, tw);
    }
}

// Forward transforms (sign -1) of NV arrays in strided order.  ZH: the
// points of the upper half (v[e], e >= E/2) are zero and are not read.
template <int N, int E, int NV, typename T, bool ZH = false>
__device__ __forceinline__ void fft_fwd(cx<T> (&v)[NV][E], int t, const Lds<T> (&lds)[NV],
                                        const Twiddles<N, E, T> &tw) {
    static_assert((N & (N - 1)) == 0 && N >= E && E >= 2, "sizes");
    static_assert(!ZH || E >= 4, "zero upper half needs E >= 4");
    fft_stages<N, E, 1, 0, NV, T, ZH>(v, t, lds, tw);
}

// The forward transform of one zero-padded array (upper half zero) times a
// power of two that f gives (see fft_stages): the values are scaled after
// the first stage's exchange.
// The result equals the transform of the scaled input exactly as long as the
// first stage's values (at most E/2 times the largest input) stay in range.
template <int N, int E, typename T, typename F>
__device__ __forceinline__ void fft_fwd_zh_scaled(cx<T> (&v)[E], int t, const Lds<T> &lds,
                                                  const Twiddles<N, E, T> &tw, F f) {
    static_assert((N & (N - 1)) == 0 && N >= E && E >= 4, "sizes");
    cx<T> vv[1][E];
    const Lds<T> l[1] = {lds};
#pragma unroll
    for (int e = 0; e < E; ++e) vv[0][e] = v[e];
    if constexpr (N == E) {   // one stage: scale the input instead
        f.pre();
        __syncthreads();
        const T sc = f.post();
#pragma unroll
        for (int e = 0; e < E; ++e) vv[0][e] = scale(vv[0][e], sc);
        fft_stages<N, E, 1, 0, 1, T, true>(vv, t, l, tw);
    } else {
        fft_stages<N, E, 1, 0, 1, T, true, F>(vv, t, l, tw, f);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vv[0][e];
}

// Inverse transforms (sign +1, unnormalised) as swap(F(swap(x))), where
// swap exchanges real and imaginary parts (swap(z) = i conj(z), so
// swap(F(swap(x))) = conj(F(conj(x)))): a register renaming, no arithmetic.
template <typename T>
__device__ __forceinline__ cx<T> swap_ri(cx<T> a) { return {a.y, a.x}; }

template <int N, int E, int NV, typename T>
__device__ __forceinline__ void fft_inv(cx<T> (&v)[NV][E], int t, const Lds<T> (&lds)[NV],
                                        const Twiddles<N, E, T> &tw) {
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int e = 0; e < E; ++e) v[a][e] = swap_ri(v[a][e]);
    fft_stages<N, E, 1, 0, NV, T>(v, t, lds, tw);
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
        for (int e = 0; e < E; ++e) v[a][e] = swap_ri(v[a][e]);
}

// Single-array forms (the copies are register renames once inlined).
template <int N, int E, typename T, bool ZH = false>
__device__ __forceinline__ void fft_fwd(cx<T> (&v)[E], int t, const Lds<T> &lds,
                                        const Twiddles<N, E, T> &tw) {
    cx<T> vv[1][E];
    const Lds<T> l[1] = {lds};
#pragma unroll
    for (int e = 0; e < E; ++e) vv[0][e] = v[e];
    fft_fwd<N, E, 1, T, ZH>(vv, t, l, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vv[0][e];
}

template <int N, int E, typename T>
__device__ __forceinline__ void fft_inv(cx<T> (&v)[E], int t, const Lds<T> &lds,
                                        const Twiddles<N, E, T> &tw) {
    cx<T> vv[1][E];
    const Lds<T> l[1] = {lds};
#pragma unroll
    for (int e = 0; e < E; ++e) vv[0][e] = v[e];
    fft_inv<N, E, 1, T>(vv, t, l, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vv[0][e];
}

}  // namespace pf
