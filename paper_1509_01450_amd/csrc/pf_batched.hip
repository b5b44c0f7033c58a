// pf_batched.hip -- the many-disk forward map: grouped launches over all disks
// of a batch, each disk at the points per thread tuned for its sizes.
//
// The disks of a batch (sizes may differ, one precision) are grouped per
// pass into classes of equal transform length and points per thread (E):
// for pass A those of the one-channel row shape of the disk's schedule, for
// pass C the two-channel one, for pass B the column shape.  Each class is
// one launch, at the tuned shape of its disk with the most units, whose
// workgroups cover every unit (G rows or G columns) of every disk of the
// class; a workgroup finds its disk by a binary search over the class's
// entry table (disk, first block), then runs the pass body of the
// single-disk kernels at that shape.  The units per workgroup change no
// arithmetic, so every disk's forces are bit for bit those of its own plan.
// Pass A of every class, then pass B, then pass C: the launch boundaries
// order the passes.  For the 64-disk workload (N_r in {256 ... 1024}, N_phi
// in {256 ... 2048}) that is 15 launches (23 when the classes also split by
// tuned G) instead of one kernel holding every size at one register budget.
//
// The tables (one descriptor per disk and the three entry tables) go to the
// device through small upload kernels that take the bytes as kernel
// arguments: no host buffer has to outlive the call and nothing waits.
// pf_forces_batched keeps them in device memory it allocates once per set of
// plans (refreshed when the field pointers change);
// pf_forces_batched_noalloc writes them, on every call, into a static device
// array of the library (for callers that cannot allocate).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "pass_bodies.hpp"
#include "rows_q.hpp"
#include "pf_batched.hpp"

namespace pf {

// ===========================================================================
// Device side
// ===========================================================================
template <typename T>
struct GDisk {
    int n_r, M, L, H, ldspec;
    T ca, c0, cn;
    const T *sigma;
    T *fr, *fp;
    cx<T> *S;
    cx2<T> *Z;     // (Zr, Zp) pairs
    const cx2<T> *spec;
    const cx<T> *twN, *twL;
    unsigned *gscale;   // the plan's FP32 scale words (nullptr in FP64)
};

// One disk in one class launch: its descriptor and its first workgroup.
struct GEntry {
    int disk;
    int first;
};

// The entry of the calling workgroup: the last one whose first block is at
// or below blockIdx.x (entries sorted by first block, n >= 1).  Wave-uniform.
__device__ __forceinline__ GEntry find_entry(const GEntry *__restrict__ ent, int n) {
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].first <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return ent[lo];
}

// Pass A (C = 1) or pass C (C = 2) of the disks of one class: G rows per
// workgroup (G = blockDim.x / (M / E)), LDS C G padded_len(M) complex.
template <typename T, int M, int E, int C>
__global__ __launch_bounds__(512) void k_grp_rows(const GDisk<T> *__restrict__ desc,
                                                  const GEntry *__restrict__ ent, int n_ent) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const GEntry en = find_entry(ent, n_ent);
    const GDisk<T> &d = desc[en.disk];
    const int unit = blockIdx.x - en.first;
    const int G = blockDim.x / (M / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        body_rows_r2c<T, M, E, 1>(unit, G, buf, d.sigma, nullptr, d.n_r, d.S, d.twN, d.gscale);
    else
        body_rows_c2r<T, M, E, 2>(unit, G, buf, reinterpret_cast<const cx<T> *>(d.Z), d.n_r,
                                  d.fr, d.fp, d.twN, d.gscale);
}

// The same for rows of N_phi = 2 Q P points (Q = 3 or 9, rows_q.hpp):
// G = blockDim.x / (P / E), LDS C G rowq_len(P, Q) complex.
template <typename T, int P, int Q, int E, int C>
__global__ __launch_bounds__(512) void k_grp_rowsq(const GDisk<T> *__restrict__ desc,
                                                   const GEntry *__restrict__ ent, int n_ent) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const GEntry en = find_entry(ent, n_ent);
    const GDisk<T> &d = desc[en.disk];
    const int unit = blockIdx.x - en.first;
    const int G = blockDim.x / (P / E);
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    if constexpr (C == 1)
        body_rows_r2cq<T, P, Q, E, 1>(unit, G, buf, d.sigma, nullptr, d.n_r, d.S, d.twN,
                                      d.gscale);
    else
        body_rows_c2rq<T, P, Q, E, 2>(unit, G, buf, reinterpret_cast<const cx<T> *>(d.Z), d.n_r,
                                      d.fr, d.fp, d.twN, d.gscale, 0);
}

// Column groups of a disk are remapped as in the single-disk kernels: a
// disk's blocks start at a multiple of 8 and run round-robin over the 8
// XCDs, and each XCD gets a contiguous range of column groups.
__device__ __forceinline__ int grp_xcd(int b, int n_groups) {
    const int per_xcd = (n_groups + 7) / 8;
    return (b & 7) * per_xcd + (b >> 3);
}

// Pass B of the disks of one class, G fixed at compile time: the transform
// buffer and the spectrum prefetch region are static LDS arrays (as the
// single-disk k_cols_fwd_pf).
template <typename T, int L, int E, int G>
__global__ __launch_bounds__(512) void k_grp_cols_pf(const GDisk<T> *__restrict__ desc,
                                                     const GEntry *__restrict__ ent, int n_ent) {
    __shared__ cx<T> fbuf[G * padded_len(L)];
    __shared__ cx2<T> spl[G * spec_prefetch_len<L, E>()];
    const GEntry en = find_entry(ent, n_ent);
    const GDisk<T> &d = desc[en.disk];
    const int n_groups = (d.H + G - 1) / G;
    const int grp = grp_xcd(blockIdx.x - en.first, n_groups);
    if (grp >= n_groups) return;   // whole workgroup leaves together
    body_cols_fwd<T, L, E, true>(grp, G, fbuf, d.S, d.Z, d.spec, d.H, d.n_r, d.n_r, d.ldspec,
                                 d.ca, d.c0, d.cn, d.twL, spl, d.gscale);
}

// Pass B for shapes without a static instance: one dynamic LDS array (FP32
// prefetches into its tail, as k_cols_fwd).
template <typename T, int L, int E>
__global__ __launch_bounds__(512) void k_grp_cols(const GDisk<T> *__restrict__ desc,
                                                  const GEntry *__restrict__ ent, int n_ent) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const GEntry en = find_entry(ent, n_ent);
    const GDisk<T> &d = desc[en.disk];
    const int G = blockDim.x / (L / E);
    const int n_groups = (d.H + G - 1) / G;
    const int grp = grp_xcd(blockIdx.x - en.first, n_groups);
    if (grp >= n_groups) return;
    cx<T> *const buf = reinterpret_cast<cx<T> *>(smem_raw);
    body_cols_fwd<T, L, E, sizeof(T) == 4>(
        grp, G, buf, d.S, d.Z, d.spec, d.H, d.n_r, d.n_r, d.ldspec, d.ca, d.c0, d.cn, d.twL,
        reinterpret_cast<cx2<T> *>(buf + (size_t)G * padded_len(L)), d.gscale);
}

// Table upload: the bytes travel as the kernel's argument.
struct UpChunk {
    static constexpr int kWords = 766;   // 3 KB of payload per launch
    unsigned int off, words;             // destination offset and length, in words
    unsigned int w[kWords];
};

__global__ __launch_bounds__(256) void k_upload(UpChunk c, unsigned int *__restrict__ dst) {
    for (unsigned int i = threadIdx.x; i < c.words; i += blockDim.x) dst[c.off + i] = c.w[i];
}

// Static device array behind pf_forces_batched_noalloc: the descriptors and
// the three entry tables of the latest call on this device.
constexpr int kNoAllocMaxDisks = 256;
constexpr size_t kNoAllocBytes = 48 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// ===========================================================================
// Host side
// ===========================================================================
// Sizes the grouped kernels instantiate.
bool batch_size_ok(const Plan &p) {
    return row_factor(p.M) != 0 && p.M >= 64 && p.M <= 2048 && p.L >= 128 && p.L <= 4096;
}

// One class launch: a kernel shape and the range [e0, e1) of its pass's
// entry table.
struct GClass {
    int pass;       // 0: pass A, 1: pass B, 2: pass C
    int n;          // transform length: M for rows, L for columns
    Shape s;
    int e0, e1;     // entries
    int blocks;     // total workgroups
};

// blocks of one disk in one pass at shape s
int disk_blocks(const Plan &p, int pass, Shape s) {
    if (pass == 1) {
        const int n_groups = (p.H + s.G - 1) / s.G;
        return (n_groups + 7) / 8 * 8;   // whole rounds of the 8 XCDs
    }
    return (p.n_r + s.G - 1) / s.G;
}

Shape pass_shape(const Plan &p, int pass) {
    return pass == 0 ? p.sched.rows : pass == 1 ? p.sched.cols : p.sched.rows2;
}

// The tables of one batch from the plans' tuned schedules: for each pass q,
// the entries ent[q n ... q n + n - 1] ordered by class (transform length,
// then points per thread), and the classes, cls[0 ... *n_cls - 1].  A class
// runs its disks with the tuned shape of its disk with the most units (rows
// or columns): the number of units per workgroup (G) changes no arithmetic
// of these forward passes, the points per thread (E) do, so disks of one
// length with the same E share a launch and every disk's result stays bit
// for bit that of its own plan.  order[n] is working space.  Allocates
// nothing (an insertion sort: batches are small).
void make_layout(const Plan *const *plans, int n, GEntry *ent, GClass *cls, int *n_cls,
                 int *order) {
    int nc = 0;
    for (int q = 0; q < 3; ++q) {
        auto key = [&](int k) {
            const Shape s = pass_shape(*plans[k], q);
            const int len = q == 1 ? plans[k]->L : plans[k]->M;
            return std::make_tuple(len, s.E, 0, k);
        };
        auto units = [&](int k) { return q == 1 ? plans[k]->H : plans[k]->n_r; };
        for (int k = 0; k < n; ++k) {
            int j = k;
            while (j > 0 && key(k) < key(order[j - 1])) {
                order[j] = order[j - 1];
                --j;
            }
            order[j] = k;
        }
        auto same = [&](int a, int b) {
            return std::get<0>(key(a)) == std::get<0>(key(b)) &&
                   std::get<1>(key(a)) == std::get<1>(key(b)) &&
                   std::get<2>(key(a)) == std::get<2>(key(b));
        };
        int i = 0;
        while (i < n) {
            int j = i;
            GClass c;
            c.pass = q;
            c.n = q == 1 ? plans[order[i]]->L : plans[order[i]]->M;
            int big = order[i];
            for (int m = i; m < n && same(order[m], order[i]); ++m)
                if (units(order[m]) > units(big)) big = order[m];
            c.s = pass_shape(*plans[big], q);
            c.e0 = q * n + i;
            int blocks = 0;
            while (j < n && same(order[j], order[i])) {
                ent[q * n + j] = GEntry{order[j], blocks};
                blocks += disk_blocks(*plans[order[j]], q, c.s);
                ++j;
            }
            c.e1 = q * n + j;
            c.blocks = blocks;
            cls[nc++] = c;
            i = j;
        }
    }
    *n_cls = nc;
}

template <typename T>
void make_desc(const Plan *const *plans, int n, const void *const *sigma, void *const *f_r,
               void *const *f_phi, GDisk<T> *desc) {
    for (int k = 0; k < n; ++k) {
        const Plan &p = *plans[k];
        GDisk<T> &d = desc[k];
        memset(&d, 0, sizeof(d));
        d.n_r = p.n_r;
        d.M = p.M;
        d.L = p.L;
        d.H = p.H;
        d.ldspec = p.ldspec;
        d.ca = (T)p.ca;
        d.c0 = (T)p.c0;
        d.cn = (T)p.cn;
        cx<T> *ws = (cx<T> *)p.ws;
        d.S = ws;
        d.Z = reinterpret_cast<cx2<T> *>(ws + (size_t)p.n_r * p.H);
        d.spec = (const cx2<T> *)p.spec;
        d.twN = (const cx<T> *)p.twN;
        d.twL = (const cx<T> *)p.twL;
        d.gscale = p.gscale;
        d.sigma = (const T *)sigma[k];
        d.fr = (T *)f_r[k];
        d.fp = (T *)f_phi[k];
    }
}

// bytes (a multiple of 4) to device memory at dst, through upload launches
int upload(const void *src, size_t bytes, void *dst, hipStream_t st) {
    const unsigned int *w = (const unsigned int *)src;
    const size_t words = bytes / 4;
    UpChunk c;
    for (size_t off = 0; off < words; off += UpChunk::kWords) {
        c.off = (unsigned int)off;
        c.words = (unsigned int)std::min<size_t>(UpChunk::kWords, words - off);
        memcpy(c.w, w + off, (size_t)c.words * 4);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, c, (unsigned int *)dst);
        PF_HIP(hipGetLastError());
    }
    return PF_OK;
}

template <typename K>
int allow_lds(K kern, size_t lds) {
    if (lds > 64 * 1024)
        PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PF_OK;
}

template <typename T>
struct GLaunch {
    const GDisk<T> *desc;
    const GEntry *ent;   // the class's entries
    int n_ent, blocks;
    hipStream_t st;

    template <int M, int E, int C>
    int rows(int G) {
        if constexpr (E <= M) {
            const size_t lds = (size_t)C * G * padded_len(M) * sizeof(cx<T>);
            int rc = allow_lds(k_grp_rows<T, M, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_grp_rows<T, M, E, C>), dim3(blocks), dim3(G * (M / E)), lds, st,
                               desc, ent, n_ent);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d points cannot take %d points per thread", M, E);
        return PF_EUNSUPPORTED;
    }
    template <int M, int C>
    int rows_e(Shape s) {
        switch (s.E) {
            case 4: return rows<M, 4, C>(s.G);
            case 8: return rows<M, 8, C>(s.G);
            case 16: return rows<M, 16, C>(s.G);
        }
        set_error("bad points per thread %d", s.E);
        return PF_EUNSUPPORTED;
    }
    template <int M>
    int rows1(Shape s) { return rows_e<M, 1>(s); }
    template <int M>
    int rows2(Shape s) { return rows_e<M, 2>(s); }
    template <int P, int Q, int E, int C>
    int rowsq(int G) {
        if constexpr (E <= P) {
            const size_t lds = (size_t)C * G * rowq_len(P, Q) * sizeof(cx<T>);
            int rc = allow_lds(k_grp_rowsq<T, P, Q, E, C>, lds);
            if (rc) return rc;
            hipLaunchKernelGGL((k_grp_rowsq<T, P, Q, E, C>), dim3(blocks), dim3(G * (P / E)), lds,
                               st, desc, ent, n_ent);
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("row transform of %d x %d points cannot take %d points per thread", Q, P, E);
        return PF_EUNSUPPORTED;
    }
    // points per thread as the standalone kernels take them: 4 or 8 (Q = 3),
    // 2 (Q = 9)
    template <int P, int Q, int C>
    int rowsq_e(Shape s) {
        if constexpr (Q == 3) {
            if (s.E == 4) return rowsq<P, 3, 4, C>(s.G);
            if (s.E == 8) return rowsq<P, 3, 8, C>(s.G);
        } else {
            if (s.E == 2) return rowsq<P, 9, 2, C>(s.G);
        }
        set_error("bad points per thread %d", s.E);
        return PF_EUNSUPPORTED;
    }
    template <int P>
    int rows1q3(Shape s) { return rowsq_e<P, 3, 1>(s); }
    template <int P>
    int rows2q3(Shape s) { return rowsq_e<P, 3, 2>(s); }
    template <int P>
    int rows1q9(Shape s) { return rowsq_e<P, 9, 1>(s); }
    template <int P>
    int rows2q9(Shape s) { return rowsq_e<P, 9, 2>(s); }
    template <int L, int E, int G>
    bool cols_pf() {
        constexpr int TH = L / E;
        if constexpr (TH >= 64 && G * TH <= 512 &&
                      (size_t)G * padded_len(L) * sizeof(cx<T>) +
                              (size_t)G * spec_prefetch_len<L, E>() * sizeof(cx2<T>) <=
                          (size_t)144 * 1024) {
            hipLaunchKernelGGL((k_grp_cols_pf<T, L, E, G>), dim3(blocks), dim3(G * TH), 0, st,
                               desc, ent, n_ent);
            return true;
        }
        return false;
    }
    template <int L, int E>
    int cols(int G) {
        if constexpr (E <= L) {
            const bool done = G == 1   ? cols_pf<L, E, 1>()
                              : G == 2 ? cols_pf<L, E, 2>()
                              : G == 4 ? cols_pf<L, E, 4>()
                                       : false;
            if (!done) {
                const size_t lds = cols_lds_bytes(L, E, G, sizeof(T) == 8, sizeof(T) == 4);
                int rc = allow_lds(k_grp_cols<T, L, E>, lds);
                if (rc) return rc;
                hipLaunchKernelGGL((k_grp_cols<T, L, E>), dim3(blocks), dim3(G * (L / E)), lds,
                                   st, desc, ent, n_ent);
            }
            PF_HIP(hipGetLastError());
            return PF_OK;
        }
        set_error("column transform of %d points cannot take %d points per thread", L, E);
        return PF_EUNSUPPORTED;
    }
    template <int L>
    int cols_e(Shape s) {
        switch (s.E) {
            case 8: return cols<L, 8>(s.G);
            case 16: return cols<L, 16>(s.G);
        }
        set_error("bad points per thread %d", s.E);
        return PF_EUNSUPPORTED;
    }
};

#define PF_SWITCH_ROWS(v, F, ...)                                                        \
    switch (v) {                                                                         \
        case 64: return F<64>(__VA_ARGS__);                                              \
        case 128: return F<128>(__VA_ARGS__);                                            \
        case 256: return F<256>(__VA_ARGS__);                                            \
        case 512: return F<512>(__VA_ARGS__);                                            \
        case 1024: return F<1024>(__VA_ARGS__);                                          \
        case 2048: return F<2048>(__VA_ARGS__);                                          \
        default: set_error("unsupported batched row length %d", v); return PF_EUNSUPPORTED; \
    }
// sub-transform lengths of the batched rows M = 3 P and M = 9 P, M in [64, 2048]
#define PF_SWITCH_P3B(v, F, ...)                                                         \
    switch (v) {                                                                         \
        case 32: return F<32>(__VA_ARGS__);                                              \
        case 64: return F<64>(__VA_ARGS__);                                              \
        case 128: return F<128>(__VA_ARGS__);                                            \
        case 256: return F<256>(__VA_ARGS__);                                            \
        case 512: return F<512>(__VA_ARGS__);                                            \
        default: set_error("unsupported batched row length 3 x %d", v); return PF_EUNSUPPORTED; \
    }
#define PF_SWITCH_P9B(v, F, ...)                                                         \
    switch (v) {                                                                         \
        case 8: return F<8>(__VA_ARGS__);                                                \
        case 16: return F<16>(__VA_ARGS__);                                              \
        case 32: return F<32>(__VA_ARGS__);                                              \
        case 64: return F<64>(__VA_ARGS__);                                              \
        case 128: return F<128>(__VA_ARGS__);                                            \
        default: set_error("unsupported batched row length 9 x %d", v); return PF_EUNSUPPORTED; \
    }
#define PF_SWITCH_COLS(v, F, ...)                                                        \
    switch (v) {                                                                         \
        case 128: return F<128>(__VA_ARGS__);                                            \
        case 256: return F<256>(__VA_ARGS__);                                            \
        case 512: return F<512>(__VA_ARGS__);                                            \
        case 1024: return F<1024>(__VA_ARGS__);                                          \
        case 2048: return F<2048>(__VA_ARGS__);                                          \
        case 4096: return F<4096>(__VA_ARGS__);                                          \
        default: set_error("unsupported batched column length %d", v); return PF_EUNSUPPORTED; \
    }

template <typename T>
int launch_class(const GClass &c, const void *desc, const GEntry *ent, hipStream_t st) {
    GLaunch<T> g{(const GDisk<T> *)desc, ent + c.e0, c.e1 - c.e0, c.blocks, st};
    if (c.pass == 1) {
        PF_SWITCH_COLS(c.n, g.template cols_e, c.s);
    }
    if (row_factor(c.n) == 3) {
        if (c.pass == 0) {
            PF_SWITCH_P3B(c.n / 3, g.template rows1q3, c.s);
        }
        PF_SWITCH_P3B(c.n / 3, g.template rows2q3, c.s);
    }
    if (row_factor(c.n) == 9) {
        if (c.pass == 0) {
            PF_SWITCH_P9B(c.n / 9, g.template rows1q9, c.s);
        }
        PF_SWITCH_P9B(c.n / 9, g.template rows2q9, c.s);
    }
    if (c.pass == 0) {
        PF_SWITCH_ROWS(c.n, g.template rows1, c.s);
    }
    PF_SWITCH_ROWS(c.n, g.template rows2, c.s);
}

// ---- pf_forces_batched: tables in device memory allocated per set of plans
struct BatchEntry {
    int n = 0, n_cls = 0;
    bool f64 = false;
    std::vector<GEntry> ent;             // 3 n
    std::vector<GClass> cls;             // up to 3 n
    std::vector<unsigned char> h_desc;   // GDisk<T>[n], as last uploaded
    void *d_tab = nullptr;               // descriptors, then the entries
    size_t desc_bytes = 0;

    void release() {
        if (d_tab) (void)hipFree(d_tab);
        d_tab = nullptr;
    }
};

std::mutex g_batch_mu;
std::map<std::vector<int64_t>, BatchEntry> g_batches;

size_t desc_size(bool f64, int n) {
    return (f64 ? sizeof(GDisk<double>) : sizeof(GDisk<float>)) * (size_t)n;
}

int check_plans(const Plan *const *plans, int n) {
    for (int k = 0; k < n; ++k) {
        if (!batch_size_ok(*plans[k])) {
            set_error("batched path needs n_phi in [128, 4096] (a power of two, or three or "
                      "nine times one) and 33 <= n_r <= 2048 "
                      "(disk %d: %d x %d)", k, plans[k]->n_r, plans[k]->n_phi);
            return PF_EUNSUPPORTED;
        }
        for (int j = 0; j < k; ++j)
            if (plans[j] == plans[k]) {
                set_error("a plan appears twice in one batch (plans own their workspace)");
                return PF_EINVAL;
            }
    }
    return PF_OK;
}

template <typename T>
int launch_classes(const GClass *cls, int n_cls, const void *desc, const GEntry *ent,
                   hipStream_t st) {
    for (int c = 0; c < n_cls; ++c) {
        const int rc = launch_class<T>(cls[c], desc, ent, st);
        if (rc) return rc;
    }
    return PF_OK;
}

}  // namespace

int batched_forces(const std::vector<const Plan *> &plans, const void *const *sigma,
                   void *const *f_r, void *const *f_phi, hipStream_t st) {
    const int n = (int)plans.size();
    const bool f64 = plans[0]->opts.dtype == PF_F64;
    int rc = check_plans(plans.data(), n);
    if (rc) return rc;
    std::vector<int64_t> key(n);
    for (int k = 0; k < n; ++k) key[k] = plans[k]->uid;
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto it = g_batches.find(key);
    if (it == g_batches.end()) {
        BatchEntry e;
        e.n = n;
        e.f64 = f64;
        e.ent.resize(3 * (size_t)n);
        e.cls.resize(3 * (size_t)n);
        std::vector<int> order(n);
        make_layout(plans.data(), n, e.ent.data(), e.cls.data(), &e.n_cls, order.data());
        e.desc_bytes = desc_size(f64, n);
        hipError_t he = hipMalloc(&e.d_tab, e.desc_bytes + e.ent.size() * sizeof(GEntry));
        if (he != hipSuccess) {
            set_error("batch table allocation failed: %s", hipGetErrorString(he));
            return PF_ENOMEM;
        }
        rc = upload(e.ent.data(), e.ent.size() * sizeof(GEntry),
                    (unsigned char *)e.d_tab + e.desc_bytes, st);
        if (rc) {
            e.release();
            return rc;
        }
        it = g_batches.emplace(key, std::move(e)).first;
    }
    BatchEntry &e = it->second;
    std::vector<unsigned char> desc(e.desc_bytes);
    if (f64)
        make_desc<double>(plans.data(), n, sigma, f_r, f_phi, (GDisk<double> *)desc.data());
    else
        make_desc<float>(plans.data(), n, sigma, f_r, f_phi, (GDisk<float> *)desc.data());
    if (desc != e.h_desc) {
        rc = upload(desc.data(), desc.size(), e.d_tab, st);
        if (rc) return rc;
        e.h_desc.swap(desc);
    }
    const GEntry *ent = (const GEntry *)((unsigned char *)e.d_tab + e.desc_bytes);
    return f64 ? launch_classes<double>(e.cls.data(), e.n_cls, e.d_tab, ent, st)
               : launch_classes<float>(e.cls.data(), e.n_cls, e.d_tab, ent, st);
}

void batched_forget(int64_t uid) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    for (auto it = g_batches.begin(); it != g_batches.end();) {
        if (std::find(it->first.begin(), it->first.end(), uid) != it->first.end()) {
            it->second.release();
            it = g_batches.erase(it);
        } else {
            ++it;
        }
    }
}

// ---- pf_forces_batched_noalloc: tables in the static device array ---------
namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};   // device address of `scratch`, per device

// The device address of the static array on the current device, looked up
// once per device with that device current (each device holds its own copy
// of the array at its own address; the array's name in host code is only a
// stand-in and is never passed to a kernel or a copy).
int scratch_address(void **out) {
    int dev = 0;
    PF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal %d beyond the library's table of 64", dev);
        return PF_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        PF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PF_OK;
}

// Host-side tables of one call, in fixed arrays (nothing allocated); calls
// from several host threads take turns on them.
struct NoAllocTables {
    unsigned char bytes[kNoAllocBytes];
    GEntry ent[3 * kNoAllocMaxDisks];
    GClass cls[3 * kNoAllocMaxDisks];
    int order[kNoAllocMaxDisks];
};
std::mutex g_na_mu;
NoAllocTables g_na;

}  // namespace

int batched_forces_noalloc(const Plan *const *plans, int n, const void *const *sigma,
                           void *const *f_r, void *const *f_phi, hipStream_t st) {
    const bool f64 = plans[0]->opts.dtype == PF_F64;
    int rc = check_plans(plans, n);
    if (rc) return rc;
    if (n > kNoAllocMaxDisks) {
        set_error("pf_forces_batched_noalloc takes at most %d disks (got %d)", kNoAllocMaxDisks,
                  n);
        return PF_EINVAL;
    }
    static_assert((size_t)kNoAllocMaxDisks * sizeof(GDisk<double>) +
                          (size_t)3 * kNoAllocMaxDisks * sizeof(GEntry) <=
                      kNoAllocBytes,
                  "static table size");
    const size_t dbytes = desc_size(f64, n);
    const size_t ebytes = (size_t)3 * n * sizeof(GEntry);
    void *dev = nullptr;
    rc = scratch_address(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(g_na_mu);
    int n_cls = 0;
    make_layout(plans, n, g_na.ent, g_na.cls, &n_cls, g_na.order);
    if (f64)
        make_desc<double>(plans, n, sigma, f_r, f_phi, (GDisk<double> *)g_na.bytes);
    else
        make_desc<float>(plans, n, sigma, f_r, f_phi, (GDisk<float> *)g_na.bytes);
    memcpy(g_na.bytes + dbytes, g_na.ent, ebytes);
    // every call rewrites the whole table (other calls on this device share
    // the array); the class launches read it in stream order
    rc = upload(g_na.bytes, dbytes + ebytes, dev, st);
    if (rc) return rc;
    const GEntry *ent = (const GEntry *)((unsigned char *)dev + dbytes);
    return f64 ? launch_classes<double>(g_na.cls, n_cls, dev, ent, st)
               : launch_classes<float>(g_na.cls, n_cls, dev, ent, st);
}

}  // namespace pf
