/*
 * pf.h -- C ABI of the log-polar thin-disk self-gravity library (libpf.so).
 *
 * The library computes the radial and azimuthal self-gravity forces F_r,
 * F_phi of an infinitesimally thin disk on a logarithmic-radial, uniform-
 * azimuth grid with the second-order method of Wang, Yen & Taam
 * (arXiv:1509.01450): the forces are three discrete convolutions per
 * component of the cell density and its two slopes with precomputed force-
 * kernel tables (Sec. 3.2.1, Eq. 26-32 and A18-A24), the tables being built
 * by the singular integration method (SIM, Sec. 4, Eq. 41-46).  The
 * convolutions run as FFTs on the GPU: zero-padded in u = ln r (no artificial
 * boundary) and periodic in phi.  G = 1 throughout (Sec. 2).
 *
 * Grid (Sec. 3.2.1, generalised to n_r x n_phi).  beta = (r_max/r_min)^(1/n_r);
 * radial cell i (0-based) spans [r_min beta^i, r_min beta^(i+1)] with centre
 * r_i = r_min beta^i (1 + beta) / 2 (the arithmetic mean of its edges);
 * dphi = 2 pi / n_phi; azimuthal cell j spans [j dphi, (j+1) dphi] with centre
 * phi_j = (j + 1/2) dphi.
 *
 * Array layout.  Every field (density, forces, their gradients) is a dense
 * row-major [n_r][n_phi] array: element (i, j) at offset i * n_phi + j, i
 * radial (inner to outer), j azimuthal.  Field pointers are DEVICE pointers
 * on the current HIP device, of the plan's precision (float for PF_F32,
 * double for PF_F64), and must not overlap one another.
 *
 * Forces follow Eq. 23-24 (and A17): F_r = -dPhi/dr (negative = inward),
 * F_phi = -(1/r) dPhi/dphi, at the cell centres.
 *
 * Ownership.  The caller owns every field buffer.  A plan owns its kernel
 * spectra, twiddle tables and workspace (device memory allocated by
 * pf_kernels_build, released by pf_plan_destroy).
 *
 * Streams.  `stream` arguments are hipStream_t values passed as void*; NULL
 * means the default stream.  Compute calls only enqueue work and return
 * without synchronising; asynchronous faults surface at the next
 * synchronising call.  A plan is not re-entrant: calls that share a plan
 * must be ordered (same stream, or synchronised), because they share the
 * plan's workspace.
 *
 * Errors.  Every call checks its arguments on the host before touching the
 * GPU; on failure nothing is enqueued, a status below is returned and
 * pf_last_error() describes it.  HIP failures return PF_EHIP with HIP's
 * message.  Functions returning a pointer return NULL on failure.
 */
#ifndef PF_H_
#define PF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_plan_s *pf_plan;

enum pf_status {
    PF_OK = 0,
    PF_EINVAL = 1,         /* bad argument                                   */
    PF_ESTATE = 2,         /* plan not built / built for another precision   */
    PF_ENOMEM = 3,         /* device or host allocation failed               */
    PF_EHIP = 4,           /* HIP runtime error                              */
    PF_ENODEV = 5,         /* no GPU device                                  */
    PF_EUNSUPPORTED = 6    /* size outside what the kernels are built for    */
};

enum pf_dtype { PF_F32 = 0, PF_F64 = 1 };

/* How the azimuthal integrals of the kernel tables are taken. */
enum pf_table_mode {
    PF_TABLE_SIM = 0,     /* n_tpz trapezoids per source cell (Sec. 4, Eq. 41-43) */
    PF_TABLE_EXACT = 1    /* the same integrals converged to rounding          */
};

/* How the singular self-cell constants K_{00} are obtained. */
enum pf_self_mode {
    PF_SELF_CARTESIAN = 0,  /* Cartesian cover of the cell (Sec. 4, Eq. 44-46) */
    PF_SELF_EXACT = 1       /* the exact integrals (principal value for       */
                            /* K^{r,0}) in local polar coordinates            */
};

/* Which force method the tables encode. */
enum pf_method {
    PF_METHOD_SIM = 0,            /* second-order method with SIM kernels (Sec. 3.2, 4) */
    PF_METHOD_PARTICLE = 1,       /* point masses sigma r dr dphi at the cell centres, */
                                  /* no self force (Eq. 35-36)                         */
    PF_METHOD_PARTICLE_PLUS = 2   /* the same plus the self-cell correction            */
                                  /* sigma K^{r,0}_00 + r delta^r K^{r,r}_00,          */
                                  /* delta^phi K^{phi,phi}_00 (Eq. 34, 37)             */
};

/* Kernel-table construction options (Sec. 4).
 *   dtype        PF_F32: FFT and spectral multiply in FP32 with FP32
 *                accumulation (tables and spectra are built in FP64 and
 *                rounded once); PF_F64: FP64 throughout.
 *   n_tpz        trapezoids per source cell in the azimuthal quadrature of
 *                the kernels (Eq. 41-43); 19 in the paper's results; 1 gives
 *                the one-trapezoid rule of Eq. 38-40.  Range 1..1024.
 *   cover_per    Cartesian cells per Delta x and per Delta y in the cover of
 *                the singular self cell (Eq. 44-45); the paper uses 10.
 *                Range 1..64.
 *   keep_tables  nonzero: keep the six FP64 kernel tables on the device so
 *                that pf_plan_tables() can return them (diagnostics).
 *   table_mode   PF_TABLE_SIM (the paper's method; n_tpz applies) or
 *                PF_TABLE_EXACT (n_tpz ignored).  K^{phi,0}, K^{phi,r} are
 *                exact in both modes (A30-A31).
 *   self_mode    PF_SELF_CARTESIAN (the paper's cover; cover_per applies) or
 *                PF_SELF_EXACT (cover_per ignored).
 *   method       PF_METHOD_SIM, PF_METHOD_PARTICLE or PF_METHOD_PARTICLE_PLUS
 *                (table_mode and n_tpz apply to SIM only; self_mode to SIM
 *                and PARTICLE_PLUS).  The forward and transpose calls are
 *                the same for every method.
 *   slope_order  how the slopes delta^r, delta^phi of Eq. 25 (the
 *                derivatives of sigma at the cell centres) are taken from
 *                the cell values: 2 = central differences (one-sided on the
 *                first and last rows); 4 = five-point central differences
 *                (radially in u = ln r) where all five points exist, the
 *                order-2 ones on the rows next to the ends.  The paper does
 *                not fix the difference; Table 1's SIM orders over
 *                N_d = 64 ... 1024 come out with order 4 (a reading).
 *                Order 4 takes the general column kernels (slower) and is
 *                refused for patch plans and batched calls.             */
typedef struct {
    int dtype;
    int n_tpz;
    int cover_per;
    int keep_tables;
    int table_mode;
    int self_mode;
    int method;
    int slope_order;
} pf_build_opts;

/* Defaults: PF_F32, n_tpz = 19, cover_per = 10, keep_tables = 0,
 * PF_TABLE_SIM, PF_SELF_CARTESIAN, PF_METHOD_SIM (the paper's method),
 * slope_order = 2. */
void pf_build_opts_default(pf_build_opts *opts);

/* Create a plan for an n_r x n_phi grid on [r_min, r_max] (Sec. 3.2.1).
 * Host only; touches no GPU.  Requirements: 4 <= n_r <= 4096;
 * n_phi a power of two in [8, 8192], three times one in [24, 6144] or nine
 * times one in [72, 4608] (the batched path: n_phi in [128, 4096]);
 * 0 < r_min < r_max, both finite.
 * Returns NULL on failure (see pf_last_error()); PF_EUNSUPPORTED-type size
 * failures are reported the same way.                                      */
pf_plan pf_plan_create(int n_r, int n_phi, double r_min, double r_max);

/* A plan for the force of one patch of a log-polar grid on another
 * (Sec. 3.2.1, Eq. 27-29: the interaction terms, and the origin terms).
 * The destination patch is the grid of pf_plan_create(n_dst, n_phi, r_min,
 * r_max); its beta and dphi define a common grid whose row k (any integer)
 * spans [r_min beta^k, r_min beta^(k+1)].  The source patch holds the rows
 * src_row0 ... src_row0 + n_src - 1 of that grid (below, above, or
 * overlapping the destination; where a source cell coincides with a
 * destination cell the singular self cell enters as in the single grid).
 * Source slopes are taken inside the source patch (one-sided on its first
 * and last rows).  wedges != 0 adds the origin wedges
 * [0, r_min beta^src_row0] x [phi_j +- dphi/2] as a further source (needs
 * src_row0 <= 0); the paper does not define their kernels: they are the
 * integrands of Eq. 30-32 and A22-A24 over the wedge with its centre at half
 * its radius (SIM and exact table modes), or a point mass sigma r_w^2
 * dphi / 2 there (particle methods), with the wedge's azimuthal slope by
 * periodic central differences and its radial slope by the one-sided
 * difference towards the first source row.  The transforms are zero-padded
 * to L >= 2 max(n_src, n_dst) along u; the kernels keep their parity in phi
 * (no azimuthal offset between the patches).  Build with pf_kernels_build;
 * pf_forces takes sigma [n_src][n_phi] and writes f_r, f_phi
 * [n_dst][n_phi] (no wedges), pf_forces_patches also the wedge densities.
 * The transpose: pf_forces_backward (no wedges) or
 * pf_forces_patches_backward (also the wedge gradient); the
 * batched path and the autotuner are for single-grid plans
 * (PF_EUNSUPPORTED).  Sizes: 4 <= n_src <= 4096,
 * |src_row0| <= 65536, n_dst and n_phi as for pf_plan_create.             */
pf_plan pf_plan_create_patches(int n_src, int src_row0, int n_dst, int n_phi, double r_min,
                               double r_max, int wedges);

/* Turn the source patch of a patch plan, and its origin wedges, by
 * src_col0 whole cells in phi: source column j' is then centred at
 * (j' + src_col0 + 1/2) dphi (Sec. 3.2.1: a constant shift between two
 * patches that share beta and dphi is a constant phase in the Fourier
 * domain; here exp(-2 pi i k src_col0 / n_phi) on azimuthal bin k, applied
 * by the forward's last pass, and its conjugate by the transpose's).  Any
 * integer (taken modulo n_phi); 0 (the default) for no turn.  Takes effect
 * for the calls enqueued after it, built or not; no rebuild.  PF_EINVAL for
 * a plan that is not a patch plan.  A shift that is not a whole number of
 * cells is not built: it would break the kernels' parity in phi.        */
int pf_plan_set_src_col0(pf_plan plan, int src_col0);

/* Build the kernel tables and their spectra on the current device
 * (Eq. 30-33, 41-46, A22-A35): one-time work, FP64 throughout, enqueued on
 * `stream` and synchronised before returning.  opts == NULL means defaults.
 * Single-grid plans then get launch shapes tuned on the device (unless
 * PF_AUTOTUNE=0; cached in PF_AUTOTUNE_CACHE, default
 * ~/.cache/pf/autotune.json).  A failed HIP call, in the build or in the
 * tuning, returns PF_EHIP (PF_ENOMEM for the workspace) with the message in
 * pf_last_error and leaves the plan unbuilt; PF_ENODEV without a device.
 * May be called again to rebuild with other options.                       */
int pf_kernels_build(pf_plan plan, const pf_build_opts *opts, void *stream);

/* Forward map (Eq. 26-29, A18-A21): sigma -> (f_r, f_phi).  sigma is the
 * cell-centre surface density; its slopes (Eq. 25) are formed inside by
 * central differences in r and phi (periodic in phi; one-sided two-point
 * differences on the first and last radial rows).  Sources are the grid
 * cells only: no mass inside r_min or outside r_max.  Asynchronous.        */
int pf_forces(pf_plan plan, const void *sigma, void *f_r, void *f_phi,
              void *stream);

/* Forward map of a patch plan: sigma_src [n_src][n_phi] (cell-centre
 * densities of the source patch) and, for plans with origin wedges,
 * sigma_wedge [n_phi] (the wedge densities at half the wedge radius; NULL
 * otherwise) -> f_r, f_phi [n_dst][n_phi] on the destination patch.
 * Asynchronous.                                                            */
int pf_forces_patches(pf_plan plan, const void *sigma_src, const void *sigma_wedge, void *f_r,
                      void *f_phi, void *stream);

/* Transpose of the forward map: g_sigma = A^T [g_fr; g_fphi], i.e. the
 * gradient of any scalar loss L(F_r, F_phi) with respect to sigma, given
 * dL/dF_r = g_fr and dL/dF_phi = g_fphi.  Overwrites g_sigma.  Not in the
 * paper: it is the exact transpose of the linear map Eq. 26-29.  Async.
 * Patch plans without origin wedges: g_fr, g_fphi [n_dst][n_phi] on the
 * destination patch, g_sigma [n_src][n_phi] on the source patch; plans with
 * wedges give PF_EINVAL (they take pf_forces_patches_backward).           */
int pf_forces_backward(pf_plan plan, const void *g_fr, const void *g_fphi,
                       void *g_sigma, void *stream);

/* Transpose of pf_forces_patches (Sec. 3.2.1 with the slopes of Eq. 25; not
 * in the paper: the exact transpose of that linear map): cotangents g_fr,
 * g_fphi [n_dst][n_phi] -> g_sigma_src [n_src][n_phi] (overwritten) and,
 * for plans with origin wedges, g_sigma_wedge [n_phi] (overwritten; NULL
 * otherwise, and then the call is pf_forces_backward).  A wedge density
 * enters its own wedge's terms and, through the wedge's radial slope (the
 * difference towards the first source row), that row too: the first source
 * row's gradient holds that share.  Device pointers, the plan's precision;
 * PF_EINVAL for a wedge argument that does not match the plan.  Two more
 * small launches than the transpose without wedges.  Asynchronous.        */
int pf_forces_patches_backward(pf_plan plan, const void *g_fr, const void *g_fphi,
                               void *g_sigma_src, void *g_sigma_wedge, void *stream);

/* Forward map for n independent disks, each with its own built plan (all of
 * one precision, sizes may differ), on `stream`: the disks are grouped per
 * pass into classes of equal transform length and tuned points per thread
 * (from each plan's pf_plan_schedule), and each class is one launch covering
 * every disk in it, at the tuned shape of its disk with the most rows or
 * columns -- pass A of all disks, then pass B, then pass C.  The results
 * equal pf_forces on each plan bit for bit (the rows or columns per
 * workgroup change no arithmetic).  Arrays sigma[k], f_r[k],
 * f_phi[k] follow plan[k]'s layout.  Sizes: n_phi in [128, 4096] (a power
 * of two, or three or nine times one) and 33 <= n_r <= 2048; other plans
 * give PF_EUNSUPPORTED.  A
 * plan may appear once per batch (PF_EINVAL otherwise).  Plans of a batch
 * share internal state: do not run two batches with common plans at once.
 * The first call for a set of plans allocates the batch's device tables
 * (released with the plans); a call whose field pointers differ from the
 * previous call's enqueues their upload (kernel arguments, nothing waits);
 * otherwise the call only enqueues the class launches (asynchronous, and it
 * may be captured into a HIP graph).  The launches read the batch's pointer table at run
 * time: a graph replay writes to the fields of the most recent call for
 * that set of plans.  1 <= n <= 4096.                                       */
int pf_forces_batched(int n, const pf_plan *plans, const void *const *sigma,
                      void *const *f_r, void *const *f_phi, void *stream);

/* pf_forces_batched for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the batch's tables (one descriptor per disk and the class entry tables)
 * go to a static 48 KiB device array of the library instead of memory
 * allocated per set of plans, rewritten by every call through upload
 * launches (kernel arguments).  Nothing is allocated and nothing waits; the
 * plans' own workspaces carry the intermediates as in pf_forces_batched.
 * Same arguments, results (bit for bit) and size limits, and at most 256
 * disks (PF_EINVAL beyond).  Each device holds one copy of the array, shared
 * by every call on that device and keeping the last call's tables: calls
 * that overlap on one device (other streams, other host threads) race and
 * must be ordered by the caller.  The current device must be the plans'.  */
int pf_forces_batched_noalloc(int n, const pf_plan *plans, const void *const *sigma,
                              void *const *f_r, void *const *f_phi, void *stream);

/* Diagnostic form of pf_forces / pf_forces_backward: the same passes, each
 * launched `reps` times back to back (1 <= reps <= 10000; every pass reads
 * only its predecessor's output, so repeats leave the result unchanged)
 * between HIP events recorded on `stream`; waits for them and writes the
 * mean duration of one launch in milliseconds to pass_ms[3] (row
 * transforms, column pass, row transforms).  backward = 0 times the forward
 * map (in0 = sigma, out0 = f_r, out1 = f_phi), backward = 1 the transpose
 * (in0 = g_fr, in1 = g_fphi, out0 = g_sigma).  Synchronous.                */
int pf_forces_timed(pf_plan plan, int backward, const void *in0, const void *in1,
                    void *out0, void *out1, int reps, void *stream, float *pass_ms);

/* Grid geometry on the host: r_centres[n_r], r_edges[n_r + 1], *dphi.
 * Any output may be NULL.                                                  */
int pf_plan_geometry(pf_plan plan, double *r_centres, double *r_edges,
                     double *dphi);

/* Self-cell kernel constants of the last build, on the host:
 * out[0] = K^{r,0}_{00}, out[1] = K^{r,r}_{00}, out[2] = K^{phi,phi}_{00}
 * (Eq. 33, 46; the other three self constants are zero by symmetry).      */
int pf_plan_selfcell(pf_plan plan, double out[3]);

/* Launch shapes chosen for the plan by the last build (autotuned unless
 * PF_AUTOTUNE=0): out[0], out[1] = points per thread and rows per workgroup
 * of the one-channel row transforms (forward pass A, transpose pass C);
 * out[2], out[3] the same for the two-channel row transforms (forward pass
 * C, transpose pass A); out[4], out[5] = points per thread and columns per
 * workgroup of the forward column pass; out[6], out[7] the same for the
 * transpose column pass.  Not in the paper: a diagnostic.                  */
int pf_plan_schedule(pf_plan plan, int out[8]);

/* Set the launch shapes of a built plan, in[8] in the layout of
 * pf_plan_schedule, in place of the autotuned or default ones (for
 * reproducible shapes without tuning, or to run a given kernel variant).
 * Each shape must fit its transform: points per thread 4, 8 or 16 for
 * power-of-two rows (rows of n_phi = 2 Q P points: 4, or 8 in FP32, for
 * Q = 3 and 2 for Q = 9, at most P) and 8 or 16 for the columns, at most
 * the transform length, at most 512 threads per workgroup, and the
 * workgroup's LDS within 144 KB; a
 * column shape also needs a power-of-two number of columns per workgroup
 * and a workgroup of whole 64-lane waves.  Otherwise PF_EINVAL (checked
 * first, against the plan's current precision, built or not) and the plan
 * keeps its shapes.  PF_ESTATE if the shapes fit but the plan is not built.
 * Not in the paper: a tuning control.                                      */
int pf_plan_set_schedule(pf_plan plan, const int in[8]);

/* Copy the six FP64 kernel tables to host memory `dst` (plan built with
 * keep_tables).  Layout: [6][2 n_r - 1][n_phi], kernels in the order
 * K^{r,0}, K^{r,r}, K^{r,phi}, K^{phi,0}, K^{phi,r}, K^{phi,phi}; row
 * m + n_r - 1 holds radial offset m = i - i' (destination minus source),
 * column n = (j - j') mod n_phi.  Patch plans: [6][n_src + n_dst - 1][n_phi],
 * row m' + n_src - 1 for the row offset m' = i - i' (the kernel of the grid
 * offset m' - src_row0).  Synchronous.                                      */
int pf_plan_tables(pf_plan plan, double *dst);

/* Release the plan and everything it owns.  NULL is ignored.              */
void pf_plan_destroy(pf_plan plan);

/* ---- Cartesian grid (Sec. 3.1) ------------------------------------------
 * The paper's uniform-grid methods, on the same three-pass FFT structure:
 * the second-order method (Eq. 9-15, A1-A13: three convolutions of the cell
 * density and its two slopes with the closed-form cell kernels A8-A13) and
 * the particle and modified particle methods (Eq. 18-21, A14-A16: point
 * masses sigma Dx Dy at the cell centres with no self force, the modified
 * method adding delta^x K^{x,x}_{00} to F^x and delta^y K^{y,y}_{00} to
 * F^y).  Grid: N_x x N_y cells of Dx by Dy; cell (i, j) at offset
 * i * N_y + j of every field, i along x.  Slopes are central differences,
 * one-sided on the first and last cell of each direction.  The convolution
 * is zero-padded in both directions (no mass outside the grid, no
 * artificial boundary).  F^x, F^y are the forces at the cell centres
 * (G = 1).  Field pointers are device pointers of the plan's precision;
 * errors, streams and ownership as for the log-polar plan.               */
typedef struct pf_cart_s *pf_cart;

enum pf_cart_method {
    PF_CART_SECOND = 0,          /* second-order method (Eq. 9-15)        */
    PF_CART_PARTICLE = 1,        /* particle method without softening     */
                                 /* and without the correction (Eq. 20)   */
    PF_CART_PARTICLE_PLUS = 2    /* modified particle method (Eq. 18-21)  */
};

/* Create a Cartesian plan; host only.  4 <= N_x, N_y <= 2048; Dx, Dy > 0
 * and finite.  NULL on failure (pf_last_error()).                        */
pf_cart pf_cart_create(int n_x, int n_y, double dx, double dy);

/* Build the kernel tables and their spectra on the current device (FP64,
 * rounded once for PF_F32), synchronised before returning.  dtype: PF_F32
 * or PF_F64; method: a pf_cart_method.  May be called again.              */
int pf_cart_build(pf_cart plan, int dtype, int method, void *stream);

/* sigma [N_x][N_y] -> f_x, f_y [N_x][N_y].  FP32 plans scale each call by
 * a power of two as the polar plans do (the forces of 2^k sigma are 2^k
 * times those of sigma wherever they are normal numbers).  Asynchronous.  */
int pf_cart_forces(pf_cart plan, const void *sigma, void *f_x, void *f_y, void *stream);

/* Diagnostic form of pf_cart_forces: each of the three passes launched
 * `reps` times back to back (1 <= reps <= 10000) between events; writes the
 * mean duration of one launch in ms to pass_ms[3].  Synchronous.          */
int pf_cart_forces_timed(pf_cart plan, const void *sigma, void *f_x, void *f_y, int reps,
                         void *stream, float *pass_ms);

/* out[0..3] = N_x, N_y, L_x, L_y (the padded transform lengths).          */
int pf_cart_geometry(pf_cart plan, int out[4]);

/* Release the plan.  NULL is ignored.                                    */
void pf_cart_destroy(pf_cart plan);

/* Per-thread description of the last failure ("" if none).                */
const char *pf_last_error(void);

/* Library version string.                                                 */
const char *pf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H_ */
