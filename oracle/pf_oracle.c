/*
 * pf_oracle.c -- plain, slow FP64 CPU reference for the log-polar thin-disk
 * self-gravity method of Wang, Yen & Taam, "Self-Gravitational Force
 * Calculation of Second Order Accuracy for Infinitesimally Thin Gaseous Disks
 * in Polar Coordinates" (arXiv:1509.01450).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the HIP
 * library.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or constant
 * generator with the library, and the library never calls it.
 *
 * What it computes (all FP64, G = 1):
 *   - the log-polar grid (Sec. 3.2.1);
 *   - the six force-kernel tables K^{r,0}, K^{r,r}, K^{r,phi}, K^{phi,0},
 *     K^{phi,r}, K^{phi,phi} (Eq. 30-32, A22-A24) as the paper's singular
 *     integration method (SIM, Sec. 4) defines them: N_tpz trapezoids in the
 *     azimuth applied to the exact radial integral (Eq. 41-43), exact double
 *     antiderivatives for K^{phi,0} and K^{phi,r} (A30-A31), and the self cell
 *     from a Cartesian cover evaluated with the Cartesian second-order method
 *     (Eq. 44-46, Eq. 9-15, A8-A13); and, as the converged reference of
 *     the same definitions, the azimuthal integrals by adaptive quadrature
 *     (table mode 1) and the self cell as the exact (principal-value)
 *     integrals in local polar coordinates;
 *   - the cell density and slopes (Eq. 25): central differences of order 2
 *     or, as an option, of order 4 where the five points exist;
 *   - the forces as the plain double sums of Eq. 27-29 and A19-A21,
 *     O((N_r N_phi)^2), at any chosen set of destination cells;
 *   - the transpose of that linear map, as a plain double sum, at any chosen
 *     set of source cells;
 *   - the particle and modified particle methods (Eq. 34-37, 56-62) as plain
 *     double sums of point masses in physical coordinates;
 *   - two patches of one log-polar grid (destination and source rows at any
 *     integer offset) and the origin wedges below the source patch, by the
 *     same direct sums (Sec. 3.2.1, Eq. 27-29), for the second-order and the
 *     particle methods;
 *   - on a uniform Cartesian grid: the six closed-form cell kernels (A8-A13),
 *     the second-order method (Eq. 9-15, A1-A7) and the particle and
 *     modified particle methods (Eq. 18-21, A14-A16) as plain double sums.
 *
 * Index conventions (0-based).  Radial cell i spans
 * [r_min beta^i, r_min beta^(i+1)], centre r_i = r_min beta^i (1+beta)/2 (the
 * arithmetic mean of its edges, Sec. 3.2.1).  Azimuthal cell j spans
 * [j dphi, (j+1) dphi], centre (j+1/2) dphi.  Tables are indexed by the offset
 * m = i - i' (destination minus source), m in [-(N_r-1), N_r-1], stored at row
 * m + N_r - 1, and by n = (j - j') mod N_phi.  With eta = rbar / r_i and
 * xi = phibar - phi_j (Eq. 33), source cell (i', j') maps to
 *   eta in [2 beta^-m/(1+beta), 2 beta^(1-m)/(1+beta)],
 *   xi  in [xi_c - dphi/2, xi_c + dphi/2],  xi_c = -n_rep dphi,
 * where n_rep is the representative of n in (-N_phi/2, N_phi/2].  The local
 * slope weight (phibar - phi_j') is xi - xi_c.
 *
 * Readings of the paper that this file takes (every one is listed in the
 * design notes of the repository):
 *   - a rectangular N_r x N_phi grid: beta from N_r, dphi from N_phi;
 *   - one grid [r_min, r_max]; mass inside r_min is not modelled;
 *   - one-sided two-point radial differences on the first and last rows;
 *   - the trapezoid rule acts on the whole azimuthal integrand including the
 *     local weight (xi - xi_c), so every table depends on (m, n) only;
 *   - H^phi_2 uses cos(xi) (the printed cos(phi) is a typo);
 *   - Cartesian grid: cell slopes by central differences, one-sided at the
 *     domain edges (the paper leaves them open); particle masses
 *     sigma Delta x Delta y;
 *   - Cartesian cover of the self cell: cell sizes Delta x / per and
 *     Delta y / per (per = 10 by default), grid aligned so the fan centre is a
 *     cell centre, a cell kept iff its centre lies in the closed fan, and the
 *     test densities' slopes taken analytically at the Cartesian centres.
 *
 * Numerical evaluation of the exact integrals.  Where the paper's closed
 * antiderivatives lose digits to cancellation (far from the singular point
 * eta = 1, xi = 0, or near xi = +-pi for H^phi_3), the same exact integral is
 * evaluated by Gauss-Legendre quadrature of an integrand that is analytic on
 * the interval; the rule used is stated at each function.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n (textbook).    */
/* ------------------------------------------------------------------------ */
#define GL_MAX 32
static double gl_x[GL_MAX + 1][GL_MAX];
static double gl_w[GL_MAX + 1][GL_MAX];
static int gl_ready = 0;

static void gl_compute(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        long double z = cosl((long double)OR_PI * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            dp = n * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            dp = n * (z * p1 - p0) / (z * z - 1);
        }
        x[i] = (double)z;
        w[i] = (double)(2 / ((1 - z * z) * dp * dp));
    }
}

static void gl_init(void)
{
    if (gl_ready) return;
#ifdef _OPENMP
#pragma omp critical(or_gl_init)
#endif
    {
        if (!gl_ready) {
            for (int n = 1; n <= GL_MAX; ++n) gl_compute(n, gl_x[n], gl_w[n]);
            gl_ready = 1;
        }
    }
}

int or_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > GL_MAX) return -1;
    gl_init();
    memcpy(x, gl_x[n], sizeof(double) * n);
    memcpy(w, gl_w[n], sizeof(double) * n);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) accumulator.                                       */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } acc_t;
static inline void acc_add(acc_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double acc_get(const acc_t *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Adaptive quadrature of K smooth functions at once: 16-point Gauss-Legendre */
/* on [a, b] against 16-point Gauss-Legendre on its two halves; an interval  */
/* is accepted when every component agrees to tol[k] (absolute), otherwise  */
/* both halves are refined.  tol[k] = rel * int |f_k| over the whole range   */
/* (a scale that does not vanish when int f_k does by symmetry).  At most    */
/* AD_BUDGET subdivisions per call: where rounding in the integrand (the    */
/* cancellation in the closed antiderivatives) keeps the two estimates from  */
/* agreeing to tol, refinement stops there.  The accepted value is the       */
/* two-half sum.                                                             */
/* ------------------------------------------------------------------------ */
#define AD_KMAX 6
#define AD_BUDGET 2000
typedef void (*ad_fn)(double x, void *ctx, double *out);

static void gl16_on(ad_fn f, void *ctx, int K, double a, double b, double *out, double *aout)
{
    const double *x = gl_x[16], *w = gl_w[16];
    const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    double v[AD_KMAX];
    for (int k = 0; k < K; ++k) {
        out[k] = 0.0;
        if (aout) aout[k] = 0.0;
    }
    for (int i = 0; i < 16; ++i) {
        f(mid + half * x[i], ctx, v);
        for (int k = 0; k < K; ++k) {
            out[k] += w[i] * v[k];
            if (aout) aout[k] += w[i] * fabs(v[k]);
        }
    }
    for (int k = 0; k < K; ++k) {
        out[k] *= half;
        if (aout) aout[k] *= fabs(half);
    }
}

static void adapt_rec(ad_fn f, void *ctx, int K, double a, double b, const double *whole,
                      const double *tol, int depth, int *budget, double *out)
{
    const double m = 0.5 * (a + b);
    double l[AD_KMAX], r[AD_KMAX];
    gl16_on(f, ctx, K, a, m, l, NULL);
    gl16_on(f, ctx, K, m, b, r, NULL);
    int ok = 1;
    for (int k = 0; k < K; ++k)
        if (fabs(l[k] + r[k] - whole[k]) > tol[k]) ok = 0;
    if (ok || depth >= 40 || *budget <= 0) {
        for (int k = 0; k < K; ++k) out[k] = l[k] + r[k];
        return;
    }
    --*budget;
    double lo[AD_KMAX], hi[AD_KMAX];
    adapt_rec(f, ctx, K, a, m, l, tol, depth + 1, budget, lo);
    adapt_rec(f, ctx, K, m, b, r, tol, depth + 1, budget, hi);
    for (int k = 0; k < K; ++k) out[k] = lo[k] + hi[k];
}

static void adapt_gl(ad_fn f, void *ctx, int K, double a, double b, double rel, double *out)
{
    double whole[AD_KMAX], mag[AD_KMAX], tol[AD_KMAX];
    gl16_on(f, ctx, K, a, b, whole, mag);
    for (int k = 0; k < K; ++k) tol[k] = rel * mag[k] + 1e-300;
    int budget = AD_BUDGET;
    adapt_rec(f, ctx, K, a, b, whole, tol, 0, &budget, out);
}

/* ------------------------------------------------------------------------ */
/* Grid (Sec. 3.2.1, generalised to N_r x N_phi).                             */
/* ------------------------------------------------------------------------ */
int or_geometry(int n_r, int n_phi, double r_min, double r_max,
                double *r_centres, double *r_edges, double *beta_out,
                double *dphi_out)
{
    if (n_r < 1 || n_phi < 1 || !(r_min > 0) || !(r_max > r_min)) return -1;
    double beta = pow(r_max / r_min, 1.0 / n_r);
    if (r_edges)
        for (int i = 0; i <= n_r; ++i) r_edges[i] = r_min * pow(beta, i);
    if (r_centres)
        for (int i = 0; i < n_r; ++i) {
            double lo = r_min * pow(beta, i), hi = r_min * pow(beta, i + 1);
            r_centres[i] = 0.5 * (lo + hi);
        }
    if (beta_out) *beta_out = beta;
    if (dphi_out) *dphi_out = 2.0 * OR_PI / n_phi;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Polar kernel pieces in eta = rbar/r_i, xi = phibar - phi_j (Eq. 33).       */
/* F(eta, xi) = sqrt(eta^2 - 2 eta cos xi + 1), written as                   */
/* sqrt((eta-1)^2 + 4 eta sin^2(xi/2)) so it keeps its digits near eta = 1.  */
/* ------------------------------------------------------------------------ */
static inline double Fpol(double eta, double s_half)
{
    double d = eta - 1.0;
    return sqrt(d * d + 4.0 * eta * s_half * s_half);
}

/* ln(eta - cos xi + F).  For eta < cos xi the sum cancels, so it is
 * rationalised with F^2 = (eta - c)^2 + sin^2 xi:
 * eta - c + F = sin^2 xi / (F - (eta - c)). */
static inline double Lpol(double eta, double c, double s, double F)
{
    double d = eta - c;
    if (d >= 0) return log(d + F);
    return log(s * s / (F - d));
}

/* Antiderivatives of Appendix A (A25-A29), each verified by differentiation:
 *   d/deta  Hr1 = eta (1 - eta c) / F^3
 *   d/deta  Hr2 = eta^2 (1 - eta c) / F^3
 *   d/deta  G3  = eta^2 sin(xi) / F^3       (H^phi_3 = xi * G3)
 *   d2/deta dxi Hp1 = eta^2 sin(xi) / F^3
 *   d2/deta dxi Hp2 = eta^3 sin(xi) / F^3                              */
static inline double Hr1(double eta, double c, double s, double sh)
{
    double F = Fpol(eta, sh);
    return -c * Lpol(eta, c, s, F) + (2.0 * c * eta - 1.0) / F;
}
static inline double Hr2(double eta, double c, double s, double sh)
{
    double F = Fpol(eta, sh);
    return -((3.0 * c * c - 1.0) * Lpol(eta, c, s, F)
             + (-6.0 * eta * c * c + 3.0 * c + eta * eta * c + eta) / F);
}
static inline double G3(double eta, double c, double s, double sh)
{
    double F = Fpol(eta, sh);
    double cot2 = (c * c) / (s * s);
    return s * ((-eta - c + eta * cot2 - c * cot2) / F + Lpol(eta, c, s, F));
}
static inline double Hp1(double eta, double xi)
{
    double c = cos(xi), s = sin(xi), sh = sin(0.5 * xi);
    double F = Fpol(eta, sh);
    return -(F + c * Lpol(eta, c, s, F));
}
static inline double Hp2(double eta, double xi)
{
    double c = cos(xi), s = sin(xi), sh = sin(0.5 * xi);
    double F = Fpol(eta, sh);
    return -((0.5 * eta + 1.5 * c) * F + (1.5 * c * c - 0.5) * Lpol(eta, c, s, F));
}

/* Exact radial integrals at a fixed azimuth xi:
 *   Ir  = int eta (1 - eta c)/F^3 deta,
 *   Ir2 = int eta^2 (1 - eta c)/F^3 deta,
 *   Iph = int eta^2 sin(xi)/F^3 deta,   over [eta_l, eta_u].
 * use_closed = 1: differences of Hr1, Hr2, G3 (valid when the radial
 * interval may contain the singular point but sin(xi) is not small);
 * use_closed = 0: 24-point Gauss-Legendre, exact to rounding whenever the
 * interval stays away from eta = 1 by a cell width (|m| >= 1) or xi is far
 * from 0. */
static void radial_integrals(double eta_l, double eta_u, double xi,
                             int use_closed, double *Ir, double *Ir2,
                             double *Iph)
{
    double c = cos(xi), s = sin(xi), sh = sin(0.5 * xi);
    if (use_closed) {
        *Ir = Hr1(eta_u, c, s, sh) - Hr1(eta_l, c, s, sh);
        *Ir2 = Hr2(eta_u, c, s, sh) - Hr2(eta_l, c, s, sh);
        *Iph = G3(eta_u, c, s, sh) - G3(eta_l, c, s, sh);
        return;
    }
    const int n = 24;
    const double *x = gl_x[n], *w = gl_w[n];
    double mid = 0.5 * (eta_u + eta_l), half = 0.5 * (eta_u - eta_l);
    double a = 0, b = 0, d = 0;
    for (int k = 0; k < n; ++k) {
        double eta = mid + half * x[k];
        double F = Fpol(eta, sh);
        double iF3 = 1.0 / (F * F * F);
        double fr = eta * (1.0 - eta * c) * iF3;
        a += w[k] * fr;
        b += w[k] * eta * fr;
        d += w[k] * eta * eta * s * iF3;
    }
    *Ir = a * half;
    *Ir2 = b * half;
    *Iph = d * half;
}

/* ------------------------------------------------------------------------ */
/* Self cell by the Cartesian cover (Sec. 4, Eq. 44-46; Fig. 1).             */
/* ------------------------------------------------------------------------ */

/* ln(y + sqrt(x^2+y^2)) with the rationalised form for y < 0. */
static inline double lnp(double y, double x, double rho)
{
    if (y >= 0) return log(y + rho);
    return log(x * x / (rho - y));
}

/* Closed-form Cartesian cell kernels (A8-A13) for one cell whose edges,
 * relative to the destination point, are [xl, xu] x [yl, yu]; (X, Y) is the
 * cell centre relative to the destination.  Output order:
 * Kx0, Kxx, Kxy, Ky0, Kyy, Kyx. */
static void cart_closed(double xl, double xu, double yl, double yu, double X,
                        double Y, double K[6])
{
    double xs[2] = {xl, xu}, ys[2] = {yl, yu};
    double ly = 0, lx = 0, ylx = 0, xly = 0, rr = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double sgn = (a == b) ? 1.0 : -1.0; /* f|^{xu}_{xl}|^{yu}_{yl} */
            double x = xs[a], y = ys[b];
            double rho = sqrt(x * x + y * y);
            double Ly = lnp(y, x, rho), Lx = lnp(x, y, rho);
            ly += sgn * Ly;
            lx += sgn * Lx;
            ylx += sgn * y * Lx;
            xly += sgn * x * Ly;
            rr += sgn * rho;
        }
    double Kx0 = -ly, Ky0 = -lx;
    K[0] = Kx0;
    K[1] = -X * Kx0 + ylx;
    K[2] = -Y * Kx0 - rr;
    K[3] = Ky0;
    K[4] = -Y * Ky0 + xly;
    K[5] = -X * Ky0 - rr;
}

/* Gauss-Legendre order for one direction of a cell of width h whose centre
 * lies at distance d from the singular point: the error of an n-point rule
 * falls like (h / 2d)^(2n); the smallest n reaching 1e-17 is taken. */
static int cover_order(double d, double h)
{
    static const int ns[6] = {2, 3, 4, 6, 8, 12};
    double q = 0.5 * h / d;
    for (int k = 0; k < 6; ++k)
        if (pow(q, 2 * ns[k]) < 1e-17) return ns[k];
    return 0;
}

/* beta, dphi: grid ratio and azimuthal width; per: Cartesian cells per
 * Delta x and per Delta y (the paper's rule of thumb is 10).
 * out[0] = K^{r,0}_{00}, out[1] = K^{r,r}_{00}, out[2] = K^{phi,phi}_{00};
 * n_cells (optional) = number of Cartesian cells inside the fan. */
int or_selfcell_cover(double beta, double dphi, int per, double *out,
                      int64_t *n_cells)
{
    if (!(beta > 1) || !(dphi > 0) || per < 1) return -1;
    gl_init();
    const double rm = 1.0;                      /* invariance, Eq. 33 */
    const double dr = 2.0 * (beta - 1.0) / (1.0 + beta);
    const double r_in = rm - 0.5 * dr, r_out = rm + 0.5 * dr;
    const double sq = sin(0.25 * dphi);
    const double Dx = r_in * 2.0 * sq * sq;      /* (r_m - dr/2)(1 - cos(dphi/2)) */
    const double Dy = dr * sin(0.5 * dphi);      /* dr sin(dphi/2)                */
    const double hx = Dx / per, hy = Dy / per;
    const double ch = cos(0.5 * dphi), shf = sin(0.5 * dphi);
    const long kx0 = (long)ceil((r_in * ch - rm) / hx);
    const long kx1 = (long)floor((r_out - rm) / hx);
    const long ky1 = (long)floor(r_out * shf / hy);
    const double rin2 = r_in * r_in, rout2 = r_out * r_out;
    const double tanh_ = shf / ch;

    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    acc_t *part = (acc_t *)calloc((size_t)nth * 3, sizeof(acc_t));
    int64_t *cnt = (int64_t *)calloc((size_t)nth, sizeof(int64_t));
    if (!part || !cnt) { free(part); free(cnt); return -2; }

#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        acc_t s1 = {0, 0}, s2 = {0, 0}, s3 = {0, 0};
        int64_t c = 0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long kx = kx0; kx <= kx1; ++kx) {
            double X = kx * hx;
            double xc = rm + X;
            for (long ky = -ky1; ky <= ky1; ++ky) {
                double Y = ky * hy;
                double yc = Y;
                double r2 = xc * xc + yc * yc;
                if (r2 < rin2 || r2 > rout2) continue;
                if (fabs(yc) > xc * tanh_) continue;
                ++c;
                double rc = sqrt(r2);
                /* test densities (Fig. 1): (a) 1, (b) rbar - r_m, (c) phibar;
                 * value and analytic slopes at the Cartesian centre */
                double sig2 = rc - rm, dx2 = xc / rc, dy2 = yc / rc;
                double sig3 = atan2(yc, xc), dx3 = -yc / r2, dy3 = xc / r2;
                double d = sqrt(X * X + Y * Y);
                int nx = 0, ny = 0;
                if (d > 4.0 * (hx > hy ? hx : hy)) {
                    nx = cover_order(d, hx);
                    ny = cover_order(d, hy);
                }
                if (nx == 0 || ny == 0) {
                    double K[6];
                    cart_closed(X - 0.5 * hx, X + 0.5 * hx, Y - 0.5 * hy,
                                Y + 0.5 * hy, X, Y, K);
                    acc_add(&s1, K[0]);
                    acc_add(&s2, sig2 * K[0] + dx2 * K[1] + dy2 * K[2]);
                    acc_add(&s3, sig3 * K[3] + dy3 * K[4] + dx3 * K[5]);
                } else {
                    /* the same cell integrals by an nx x ny Gauss rule of the
                     * kernel times the cell's linear density (Eq. 8) */
                    double a1 = 0, a2 = 0, a3 = 0;
                    for (int p = 0; p < nx; ++p) {
                        double u = 0.5 * hx * gl_x[nx][p];
                        double xb = X + u;
                        double t1 = 0, t2 = 0, t3 = 0;
                        for (int q = 0; q < ny; ++q) {
                            double v = 0.5 * hy * gl_x[ny][q];
                            double yb = Y + v;
                            double rho2 = xb * xb + yb * yb;
                            double ir3 = 1.0 / (rho2 * sqrt(rho2));
                            double wq = gl_w[ny][q];
                            t1 += wq * xb * ir3;
                            t2 += wq * xb * ir3 * (sig2 + dx2 * u + dy2 * v);
                            t3 += wq * yb * ir3 * (sig3 + dx3 * u + dy3 * v);
                        }
                        double wp = gl_w[nx][p];
                        a1 += wp * t1;
                        a2 += wp * t2;
                        a3 += wp * t3;
                    }
                    double jac = 0.25 * hx * hy;
                    acc_add(&s1, a1 * jac);
                    acc_add(&s2, a2 * jac);
                    acc_add(&s3, a3 * jac);
                }
            }
        }
        part[3 * tid + 0] = s1;
        part[3 * tid + 1] = s2;
        part[3 * tid + 2] = s3;
        cnt[tid] = c;
    }
    acc_t t[3] = {{0, 0}, {0, 0}, {0, 0}};
    int64_t total = 0;
    for (int k = 0; k < nth; ++k) {
        for (int q = 0; q < 3; ++q) {
            acc_add(&t[q], part[3 * k + q].s);
            acc_add(&t[q], part[3 * k + q].c);
        }
        total += cnt[k];
    }
    out[0] = acc_get(&t[0]);             /* K^{r,0}_{00}           */
    out[1] = acc_get(&t[1]) / rm;        /* K^{r,r}_{00}  (Eq. 46) */
    out[2] = acc_get(&t[2]);             /* K^{phi,phi}_{00}       */
    if (n_cells) *n_cells = total;
    free(part);
    free(cnt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Self cell as the exact integrals (principal value for K^{r,0}), in local    */
/* polar coordinates (rho, t) about the cell centre x = (1, 0), xbar - x =   */
/* rho (cos t, sin t), rho up to the fan's boundary rho_max(t):              */
/*   K^{r,0}_{00}     = int cos t ln rho_max(t) dt                           */
/*   K^{r,r}_{00}     = int cos t int_0^rho_max (|xbar| - 1) / rho drho dt    */
/*   K^{phi,phi}_{00} = int sin t int_0^rho_max xi(xbar) / rho drho dt,       */
/* xi(xbar) the azimuth of xbar.  (From Eq. 30-32 with eta deta dxi = dA,     */
/* (1 - eta cos xi) = -rho cos t, eta sin xi = rho sin t, F = rho; the        */
/* log(0) part of K^{r,0} cancels over the full circle.)  The t-integrals     */
/* are split at the four corner directions, where rho_max has kinks, and at */
/* the two directions tangent to the inner circle, where the ray stops      */
/* meeting the inner arc (rho_max jumps there when the tangent point lies on */
/* the cell's inner arc).                                                    */
/* ------------------------------------------------------------------------ */
typedef struct { double r_in, r_out, a; } fan_t;

static double fan_rho_max(const fan_t *f, double t)
{
    const double c = cos(t), s = sin(t);
    double best = -c + sqrt(c * c + f->r_out * f->r_out - 1.0);
    const double disc = c * c - (1.0 - f->r_in * f->r_in);
    if (disc >= 0.0) {
        const double q = sqrt(disc);
        if (-c - q > 0.0 && -c - q < best) best = -c - q;
        if (-c + q > 0.0 && -c + q < best) best = -c + q;
    }
    for (int sg = -1; sg <= 1; sg += 2) {
        const double sa = sg * f->a;
        const double den = s * cos(sa) - c * sin(sa);
        if (den != 0.0) {
            const double rr = sin(sa) / den;
            if (rr > 0.0 && rr < best) best = rr;
        }
    }
    return best;
}

static void pv_integrand(double t, void *vctx, double *out)
{
    const fan_t *f = (const fan_t *)vctx;
    const double c = cos(t), s = sin(t), rm = fan_rho_max(f, t);
    const int n = 24;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < n; ++k) {
        const double rho = 0.5 * rm * (1.0 + gl_x[n][k]);
        const double X = 1.0 + rho * c, Y = rho * s;
        const double R = hypot(X, Y);
        /* (|xbar| - 1)/rho = (2c + rho)/(|xbar| + 1), no cancellation */
        a += gl_w[n][k] * (2.0 * c + rho) / (R + 1.0);
        b += gl_w[n][k] * atan2(Y, X) / rho;
    }
    out[0] = c * log(rm);
    out[1] = c * 0.5 * rm * a;
    out[2] = s * 0.5 * rm * b;
}

int or_selfcell_pv(double beta, double dphi, double *out)
{
    if (!(beta > 1.0) || !(dphi > 0.0) || dphi >= OR_PI || !out) return -1;
    gl_init();
    fan_t f;
    f.r_in = 2.0 / (1.0 + beta);
    f.r_out = 2.0 * beta / (1.0 + beta);
    f.a = 0.5 * dphi;
    double brk[8];
    int nb = 0;
    brk[nb++] = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int sg = -1; sg <= 1; sg += 2) {
            const double R = i ? f.r_out : f.r_in, sa = sg * f.a;
            double t = atan2(R * sin(sa), R * cos(sa) - 1.0);
            if (t < 0.0) t += 2.0 * OR_PI;
            brk[nb++] = t;
        }
    for (int sg = -1; sg <= 1; sg += 2) {
        /* tangent point T of the inner circle seen from (1, 0): T_x = r_in^2 */
        double t = atan2(sg * f.r_in * sqrt(1.0 - f.r_in * f.r_in), f.r_in * f.r_in - 1.0);
        if (t < 0.0) t += 2.0 * OR_PI;
        brk[nb++] = t;
    }
    brk[nb++] = 2.0 * OR_PI;
    /* sort the break points */
    for (int i = 1; i < nb; ++i)
        for (int j = i; j > 0 && brk[j] < brk[j - 1]; --j) {
            double x = brk[j]; brk[j] = brk[j - 1]; brk[j - 1] = x;
        }
    double acc[3] = {0, 0, 0};
    for (int i = 0; i + 1 < nb; ++i) {
        if (brk[i + 1] - brk[i] <= 0.0) continue;
        double v[3];
        adapt_gl(pv_integrand, &f, 3, brk[i], brk[i + 1], 1e-15, v);
        for (int k = 0; k < 3; ++k) acc[k] += v[k];
    }
    for (int k = 0; k < 3; ++k) out[k] = acc[k];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One table entry (all six kernels) for offset (m, n_rep).                   */
/* Output order: r0, rr, rphi, phi0, phir, phiphi.                            */
/* self = K^{r,0}_{00}, K^{r,r}_{00}, K^{phi,phi}_{00} (used at m = n = 0).   */
/* ------------------------------------------------------------------------ */
/* integrand of the four azimuthal integrals at xi (EXACT mode) */
typedef struct { double eta_l, eta_u, rho, xic; int m; } xi_ctx;

static void xi_integrand(double xi, void *vctx, double *out)
{
    const xi_ctx *c = (const xi_ctx *)vctx;
    int closed = (c->m == 0) && (fabs(xi) < 0.5 * OR_PI);
    double Ir, Ir2, Iph;
    radial_integrals(c->eta_l, c->eta_u, xi, closed, &Ir, &Ir2, &Iph);
    double wl = xi - c->xic;
    out[0] = Ir;
    out[1] = Ir2 - c->rho * Ir;
    out[2] = wl * Ir;
    out[3] = wl * Iph;
}

/* table_mode 0: SIM, n_tpz trapezoids in xi (Eq. 41-43); 1: the same
 * azimuthal integrals converged (adaptive Gauss-Legendre, split at xi = 0). */
static void table_entry(double beta, double dphi, int n_tpz, int table_mode, int m, int nrep,
                        const double self[3], double T[6])
{
    if (m == 0 && nrep == 0) {
        T[0] = self[0];
        T[1] = self[1];
        T[2] = 0.0; /* odd integrand about the cell centre (Eq. 37 text) */
        T[3] = 0.0;
        T[4] = 0.0;
        T[5] = self[2];
        return;
    }
    const double rho = pow(beta, -m);                  /* r_i' / r_i     */
    const double eta_l = 2.0 * rho / (1.0 + beta);
    const double eta_u = beta * eta_l;
    const double xic = -nrep * dphi;
    double r0 = 0, rr = 0, rph = 0, pp = 0;
    if (table_mode == 1) {
        xi_ctx c = {eta_l, eta_u, rho, xic, m};
        double lo = xic - 0.5 * dphi, hi = xic + 0.5 * dphi, v[4];
        if (lo < 0.0 && hi > 0.0) {   /* peak (or singular point) at xi = 0 */
            double v2[4];
            adapt_gl(xi_integrand, &c, 4, lo, 0.0, 4e-15, v);
            adapt_gl(xi_integrand, &c, 4, 0.0, hi, 4e-15, v2);
            for (int k = 0; k < 4; ++k) v[k] += v2[k];
        } else {
            adapt_gl(xi_integrand, &c, 4, lo, hi, 4e-15, v);
        }
        r0 = v[0];
        rr = v[1];
        rph = v[2];
        pp = v[3];
    } else {
        /* Eq. 41-43 with the weight (xi - xi_c) inside the trapezoid */
        const double dth = dphi / n_tpz;
        for (int k = 0; k <= n_tpz; ++k) {
            double xi = xic - 0.5 * dphi + k * dth;
            double wk = (k == 0 || k == n_tpz) ? 0.5 * dth : dth;
            int closed = (m == 0) && (fabs(xi) < 0.5 * OR_PI);
            double Ir, Ir2, Iph;
            radial_integrals(eta_l, eta_u, xi, closed, &Ir, &Ir2, &Iph);
            double wl = xi - xic;
            r0 += wk * Ir;
            rr += wk * (Ir2 - rho * Ir);
            rph += wk * wl * Ir;
            pp += wk * wl * Iph;
        }
    }
    T[0] = -r0;
    T[1] = -rr;
    T[2] = -rph;
    T[5] = pp;

    /* K^{phi,0}, K^{phi,r}: exact double integrals (A30-A31) */
    double xl = xic - 0.5 * dphi, xu = xic + 0.5 * dphi;
    if (m == 0) {
        double p1 = Hp1(eta_u, xu) - Hp1(eta_u, xl) - Hp1(eta_l, xu) + Hp1(eta_l, xl);
        double p2 = Hp2(eta_u, xu) - Hp2(eta_u, xl) - Hp2(eta_l, xu) + Hp2(eta_l, xl);
        T[3] = p1;
        T[4] = p2 - rho * p1;
    } else {
        /* exact azimuthal integral: int eta^2 sin xi / F^3 dxi = -eta / F,
         * and 1/F_l - 1/F_u = 4 eta sin(xi_c) sin(dphi/2) /
         * (F_l F_u (F_l + F_u)); then 24-point Gauss-Legendre in eta */
        const int n = 24;
        double mid = 0.5 * (eta_u + eta_l), half = 0.5 * (eta_u - eta_l);
        double shl = sin(0.5 * xl), shu = sin(0.5 * xu);
        double num = 4.0 * sin(xic) * sin(0.5 * dphi);
        double a = 0, b = 0;
        for (int k = 0; k < n; ++k) {
            double eta = mid + half * gl_x[n][k];
            double Fl = Fpol(eta, shl), Fu = Fpol(eta, shu);
            double D = num * eta / (Fl * Fu * (Fl + Fu));
            a += gl_w[n][k] * eta * D;
            b += gl_w[n][k] * eta * (eta - rho) * D;
        }
        T[3] = a * half;
        T[4] = b * half;
    }
}

int or_table_entry(int n_r, int n_phi, double r_min, double r_max, int n_tpz,
                   int table_mode, int m, int nrep, const double *self, double *T)
{
    double beta, dphi;
    if (or_geometry(n_r, n_phi, r_min, r_max, NULL, NULL, &beta, &dphi)) return -1;
    if ((table_mode == 0 && n_tpz < 1) || table_mode < 0 || table_mode > 1) return -1;
    gl_init();
    table_entry(beta, dphi, n_tpz, table_mode, m, nrep, self, T);
    return 0;
}

/* All six tables, each (2 N_r - 1) x N_phi, row m + N_r - 1, column n.
 * Entries are computed for n_rep in [0, N_phi/2] and mirrored to -n_rep by
 * the parity of each integrand in xi (even: r0, rr, phiphi; odd: rphi,
 * phi0, phir), which holds for every cell of the periodic grid. */
int or_tables(int n_r, int n_phi, double r_min, double r_max, int n_tpz,
              int table_mode, const double *self, double *T)
{
    double beta, dphi;
    if (or_geometry(n_r, n_phi, r_min, r_max, NULL, NULL, &beta, &dphi)) return -1;
    if ((table_mode == 0 && n_tpz < 1) || table_mode < 0 || table_mode > 1 || (n_phi % 2) != 0)
        return -1;
    gl_init();
    const long rows = 2L * n_r - 1;
    const long plane = rows * (long)n_phi;
    static const double par[6] = {1, 1, -1, -1, -1, 1};
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
#endif
    for (long row = 0; row < rows; ++row)
        for (int nrep = 0; nrep <= n_phi / 2; ++nrep) {
            int m = (int)(row - (n_r - 1));
            double t[6];
            table_entry(beta, dphi, n_tpz, table_mode, m, nrep, self, t);
            long cpos = nrep, cneg = (n_phi - nrep) % n_phi;
            for (int k = 0; k < 6; ++k) {
                T[k * plane + row * n_phi + cpos] = t[k];
                if (cneg != cpos) T[k * plane + row * n_phi + cneg] = par[k] * t[k];
            }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Density channels: the slopes delta^r = d sigma/dr and delta^phi =          */
/* d sigma/dphi at the cell centres that Eq. 25 takes, from the cell values.  */
/* order 2: central differences (P. 5.3), one-sided on the first and last     */
/*   rows: delta^r[i] = (s[i+1] - s[i-1]) / (r[i+1] - r[i-1]),                */
/*   delta^phi[j] = (s[j+1] - s[j-1]) / (2 dphi) (periodic in phi).           */
/* order 4: the five-point central differences where all five points exist:  */
/*   delta^phi[j] = (s[j-2] - 8 s[j-1] + 8 s[j+1] - s[j+2]) / (12 dphi), and  */
/*   on the rows 2 .. n_r - 3, in u = ln r (the grid is uniform in u,        */
/*   u[i+1] - u[i] = ln beta) and d/dr = (1/r) d/du:                         */
/*   delta^r[i] = (s[i-2] - 8 s[i-1] + 8 s[i+1] - s[i+2]) / (12 ln(beta) r[i]);*/
/*   rows 1 and n_r - 2 keep the order-2 central difference, rows 0 and       */
/*   n_r - 1 the one-sided one.                                              */
/* sigma, dr, dph are [n_r][n_phi].                                           */
/* ------------------------------------------------------------------------ */
/* coefficient of sigma[i] in delta^r[i2] */
static double dr_coef(int n_r, const double *rc, int order, int i2, int i)
{
    if (i2 == 0) {
        double inv = 1.0 / (rc[1] - rc[0]);
        return i == 1 ? inv : (i == 0 ? -inv : 0.0);
    }
    if (i2 == n_r - 1) {
        double inv = 1.0 / (rc[n_r - 1] - rc[n_r - 2]);
        return i == n_r - 1 ? inv : (i == n_r - 2 ? -inv : 0.0);
    }
    if (order == 4 && i2 >= 2 && i2 <= n_r - 3) {
        double h = 1.0 / (12.0 * log(rc[1] / rc[0]) * rc[i2]);
        int d = i - i2;
        return d == -2 ? h : d == -1 ? -8.0 * h : d == 1 ? 8.0 * h : d == 2 ? -h : 0.0;
    }
    double inv = 1.0 / (rc[i2 + 1] - rc[i2 - 1]);
    return i == i2 + 1 ? inv : (i == i2 - 1 ? -inv : 0.0);
}

/* coefficient of sigma[j2 + d] in delta^phi[j2] (d taken mod n_phi) */
static double dp_coef(int order, double dphi, int d)
{
    if (order == 4) {
        double h = 1.0 / (12.0 * dphi);
        return d == -2 ? h : d == -1 ? -8.0 * h : d == 1 ? 8.0 * h : d == 2 ? -h : 0.0;
    }
    return d == 1 ? 0.5 / dphi : d == -1 ? -0.5 / dphi : 0.0;
}

int or_channels_o(int n_r, int n_phi, const double *r_c, double dphi, int order,
                  const double *sigma, double *dr, double *dph)
{
    if (n_r < 2 || n_phi < 3 || (order != 2 && order != 4)) return -1;
    if (order == 4 && (n_r < 4 || n_phi < 5)) return -1;
    for (int i = 0; i < n_r; ++i)
        for (int j = 0; j < n_phi; ++j) {
            double a = 0.0, b = 0.0;
            for (int d = -2; d <= 2; ++d) {
                int jj = ((j + d) % n_phi + n_phi) % n_phi, ii = i + d;
                a += dp_coef(order, dphi, d) * sigma[(long)i * n_phi + jj];
                if (ii >= 0 && ii < n_r)
                    b += dr_coef(n_r, r_c, order, i, ii) * sigma[(long)ii * n_phi + j];
            }
            dph[(long)i * n_phi + j] = a;
            dr[(long)i * n_phi + j] = b;
        }
    return 0;
}

int or_channels(int n_r, int n_phi, const double *r_c, double dphi,
                const double *sigma, double *dr, double *dph)
{
    return or_channels_o(n_r, n_phi, r_c, dphi, 2, sigma, dr, dph);
}

/* ------------------------------------------------------------------------ */
/* Forward direct sums (Eq. 27-29 and A19-A21) at chosen destinations.        */
/* dest: n_dest flat indices i*n_phi + j (NULL = every cell, in order).       */
/* ------------------------------------------------------------------------ */
int or_forward_o(int n_r, int n_phi, double r_min, double r_max, int order, const double *T,
                 const double *sigma, const int64_t *dest, int64_t n_dest,
                 double *f_r, double *f_phi)
{
    double beta, dphi;
    double *rc = (double *)malloc(sizeof(double) * n_r);
    if (!rc) return -2;
    if (or_geometry(n_r, n_phi, r_min, r_max, rc, NULL, &beta, &dphi)) { free(rc); return -1; }
    const long N = (long)n_r * n_phi;
    double *dr = (double *)malloc(sizeof(double) * N);
    double *dp = (double *)malloc(sizeof(double) * N);
    int *live = (int *)malloc(sizeof(int) * n_r);
    if (!dr || !dp || !live) { free(rc); free(dr); free(dp); free(live); return -2; }
    if (or_channels_o(n_r, n_phi, rc, dphi, order, sigma, dr, dp)) {
        free(rc); free(dr); free(dp); free(live); return -1;
    }
    /* rows whose three channels are all zero contribute nothing */
    for (int i = 0; i < n_r; ++i) {
        live[i] = 0;
        for (int j = 0; j < n_phi; ++j) {
            long p = (long)i * n_phi + j;
            if (sigma[p] != 0 || dr[p] != 0 || dp[p] != 0) { live[i] = 1; break; }
        }
    }
    const long rows = 2L * n_r - 1;
    const long plane = rows * (long)n_phi;
    const double *Tr0 = T, *Trr = T + plane, *Trp = T + 2 * plane;
    const double *Tp0 = T + 3 * plane, *Tpr = T + 4 * plane, *Tpp = T + 5 * plane;
    const int64_t nd = dest ? n_dest : (int64_t)N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t q = 0; q < nd; ++q) {
        long d = dest ? (long)dest[q] : (long)q;
        int i = (int)(d / n_phi), j = (int)(d % n_phi);
        acc_t a0 = {0, 0}, ar = {0, 0}, ap = {0, 0};  /* F^{r,0}+F^{r,phi}, F^{r,r} */
        acc_t b0 = {0, 0}, br = {0, 0}, bp = {0, 0};
        for (int ip = 0; ip < n_r; ++ip) {
            if (!live[ip]) continue;
            long row = (long)(i - ip) + (n_r - 1);
            const double *t0 = Tr0 + row * n_phi, *tr = Trr + row * n_phi, *tp = Trp + row * n_phi;
            const double *u0 = Tp0 + row * n_phi, *ur = Tpr + row * n_phi, *up = Tpp + row * n_phi;
            const double *sg = sigma + (long)ip * n_phi, *gr = dr + (long)ip * n_phi,
                         *gp = dp + (long)ip * n_phi;
            double x0 = 0, xr = 0, xp = 0, y0 = 0, yr = 0, yp = 0;
            for (int jp = 0; jp < n_phi; ++jp) {
                int n = j - jp;
                if (n < 0) n += n_phi;
                x0 += sg[jp] * t0[n];
                xr += gr[jp] * tr[n];
                xp += gp[jp] * tp[n];
                y0 += sg[jp] * u0[n];
                yr += gr[jp] * ur[n];
                yp += gp[jp] * up[n];
            }
            acc_add(&a0, x0); acc_add(&ar, xr); acc_add(&ap, xp);
            acc_add(&b0, y0); acc_add(&br, yr); acc_add(&bp, yp);
        }
        /* F = F^{.,0} + r_i [sum delta^r K^{.,r}] + F^{.,phi}  (Eq. 26-29) */
        f_r[q] = acc_get(&a0) + rc[i] * acc_get(&ar) + acc_get(&ap);
        f_phi[q] = acc_get(&b0) + rc[i] * acc_get(&br) + acc_get(&bp);
    }
    free(rc); free(dr); free(dp); free(live);
    return 0;
}

int or_forward(int n_r, int n_phi, double r_min, double r_max, const double *T,
               const double *sigma, const int64_t *dest, int64_t n_dest,
               double *f_r, double *f_phi)
{
    return or_forward_o(n_r, n_phi, r_min, r_max, 2, T, sigma, dest, n_dest, f_r, f_phi);
}

/* ------------------------------------------------------------------------ */
/* Transpose of the forward map, as a plain double sum, at chosen sources.    */
/* Given cotangents v_r, v_phi on every destination, returns                  */
/*   g[p] = sum_q v_r[q] dF_r[q]/dsigma[p] + v_phi[q] dF_phi[q]/dsigma[p].    */
/* ------------------------------------------------------------------------ */
static void adj_u(int n_r, int n_phi, const double *rc, const double *T,
                  const double *v_r, const double *v_p, int ip, int jp,
                  double *us, double *ug, double *uh)
{
    const long rows = 2L * n_r - 1;
    const long plane = rows * (long)n_phi;
    acc_t s = {0, 0}, g = {0, 0}, h = {0, 0};
    for (int i = 0; i < n_r; ++i) {
        long row = (long)(i - ip) + (n_r - 1);
        const double *t0 = T + row * n_phi, *tr = T + plane + row * n_phi,
                     *tp = T + 2 * plane + row * n_phi;
        const double *u0 = T + 3 * plane + row * n_phi, *ur = T + 4 * plane + row * n_phi,
                     *up = T + 5 * plane + row * n_phi;
        const double *vr = v_r + (long)i * n_phi, *vp = v_p + (long)i * n_phi;
        double xs = 0, xg = 0, xh = 0;
        for (int j = 0; j < n_phi; ++j) {
            int n = j - jp;
            if (n < 0) n += n_phi;
            xs += vr[j] * t0[n] + vp[j] * u0[n];
            xg += vr[j] * tr[n] + vp[j] * ur[n];
            xh += vr[j] * tp[n] + vp[j] * up[n];
        }
        acc_add(&s, xs);
        acc_add(&g, rc[i] * xg);
        acc_add(&h, xh);
    }
    *us = acc_get(&s);
    *ug = acc_get(&g);
    *uh = acc_get(&h);
}

int or_adjoint_o(int n_r, int n_phi, double r_min, double r_max, int order, const double *T,
                 const double *v_r, const double *v_phi, const int64_t *src,
                 int64_t n_src, double *g)
{
    double beta, dphi;
    double *rc = (double *)malloc(sizeof(double) * n_r);
    if (!rc) return -2;
    if (or_geometry(n_r, n_phi, r_min, r_max, rc, NULL, &beta, &dphi)) { free(rc); return -1; }
    if (n_r < 2 || n_phi < 3 || (order != 2 && order != 4) ||
        (order == 4 && (n_r < 4 || n_phi < 5))) { free(rc); return -1; }
    const long N = (long)n_r * n_phi;
    const int64_t ns = src ? n_src : (int64_t)N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < ns; ++q) {
        long p = src ? (long)src[q] : (long)q;
        int ip = (int)(p / n_phi), jp = (int)(p % n_phi);
        double us, ug, uh, tot = 0;
        adj_u(n_r, n_phi, rc, T, v_r, v_phi, ip, jp, &us, &ug, &uh);
        tot = us;
        /* radial slope channel: sum over i2 of coef(i2, ip) * u_g(i2, jp) */
        for (int i2 = ip - 2; i2 <= ip + 2; ++i2) {
            if (i2 < 0 || i2 >= n_r) continue;
            double cf = dr_coef(n_r, rc, order, i2, ip);
            if (cf == 0.0) continue;
            double a, b, c;
            adj_u(n_r, n_phi, rc, T, v_r, v_phi, i2, jp, &a, &b, &c);
            tot += cf * b;
        }
        /* azimuthal slope channel: sigma[jp] enters delta^phi[jp - d] with
         * the coefficient of offset d, so it meets u_h at jp - d */
        for (int d = -2; d <= 2; ++d) {
            double cf = dp_coef(order, dphi, d);
            if (cf == 0.0) continue;
            int j2 = ((jp - d) % n_phi + n_phi) % n_phi;
            double a, b, h;
            adj_u(n_r, n_phi, rc, T, v_r, v_phi, ip, j2, &a, &b, &h);
            tot += cf * h;
        }
        g[q] = tot;
    }
    free(rc);
    return 0;
}

int or_adjoint(int n_r, int n_phi, double r_min, double r_max, const double *T,
               const double *v_r, const double *v_phi, const int64_t *src,
               int64_t n_src, double *g)
{
    return or_adjoint_o(n_r, n_phi, r_min, r_max, 2, T, v_r, v_phi, src, n_src, g);
}

/* ------------------------------------------------------------------------ */
/* Particle and modified particle methods in polar coordinates (Eq. 34-37,   */
/* 56-62), as plain double sums in physical coordinates.  Each source cell is */
/* a point mass Mbar = sigma r_i' dr_i' dphi at its centre (with arithmetic  */
/* centres this is the density times the exact polar cell area), and a cell  */
/* feels no force from itself.  The force of a point mass M at (r', phi') on  */
/* (r_i, phi_j) is M (r' cos d - r_i, r' sin d) / D^(3/2) in (r-hat, phi-hat), */
/* d = phi' - phi_j, D = (r_i - r')^2 + 4 r_i r' sin^2(d/2).                 */
/* plus = 1 adds the self-cell correction of the modified method:             */
/*   F^{r,corr}   = sigma K^{r,0}_{00} + r_i delta^r K^{r,r}_{00},           */
/*   F^{phi,corr} = delta^phi K^{phi,phi}_{00}                               */
/* (K^{r,phi}_{00}, K^{phi,0}_{00}, K^{phi,r}_{00} vanish by symmetry);      */
/* self = K^{r,0}_{00}, K^{r,r}_{00}, K^{phi,phi}_{00}.                       */
/* ------------------------------------------------------------------------ */
int or_forward_particle_o(int n_r, int n_phi, double r_min, double r_max, int plus, int order,
                          const double *self, const double *sigma, const int64_t *dest,
                          int64_t n_dest, double *f_r, double *f_phi)
{
    double beta, dphi;
    double *rc = (double *)malloc(sizeof(double) * n_r);
    double *re = (double *)malloc(sizeof(double) * (n_r + 1));
    if (!rc || !re) { free(rc); free(re); return -2; }
    if (or_geometry(n_r, n_phi, r_min, r_max, rc, re, &beta, &dphi)) {
        free(rc); free(re); return -1;
    }
    const long N = (long)n_r * n_phi;
    double *dr = (double *)malloc(sizeof(double) * N);
    double *dp = (double *)malloc(sizeof(double) * N);
    double *mass = (double *)malloc(sizeof(double) * N);
    if (!dr || !dp || !mass) { free(rc); free(re); free(dr); free(dp); free(mass); return -2; }
    if (or_channels_o(n_r, n_phi, rc, dphi, order, sigma, dr, dp)) {
        free(rc); free(re); free(dr); free(dp); free(mass); return -1;
    }
    for (int i = 0; i < n_r; ++i) {
        const double area = 0.5 * (re[i + 1] * re[i + 1] - re[i] * re[i]) * dphi;
        for (int j = 0; j < n_phi; ++j) mass[(long)i * n_phi + j] = sigma[(long)i * n_phi + j] * area;
    }
    const long nd = dest ? (long)n_dest : N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long q = 0; q < nd; ++q) {
        const long cell = dest ? (long)dest[q] : q;
        const int i = (int)(cell / n_phi), j = (int)(cell % n_phi);
        acc_t ar = {0, 0}, ap = {0, 0};
        for (int i2 = 0; i2 < n_r; ++i2) {
            const double r2 = rc[i2];
            for (int j2 = 0; j2 < n_phi; ++j2) {
                if (i2 == i && j2 == j) continue;
                const double M = mass[(long)i2 * n_phi + j2];
                if (M == 0.0) continue;
                const double d = (j2 - j) * dphi;
                const double sh = sin(0.5 * d);
                const double D = (rc[i] - r2) * (rc[i] - r2) + 4.0 * rc[i] * r2 * sh * sh;
                const double w = M / (D * sqrt(D));
                acc_add(&ar, w * (r2 * cos(d) - rc[i]));
                acc_add(&ap, w * r2 * sin(d));
            }
        }
        double fr = acc_get(&ar), fp = acc_get(&ap);
        if (plus) {
            fr += sigma[cell] * self[0] + rc[i] * dr[cell] * self[1];
            fp += dp[cell] * self[2];
        }
        f_r[q] = fr;
        f_phi[q] = fp;
    }
    free(rc); free(re); free(dr); free(dp); free(mass);
    return 0;
}

int or_forward_particle(int n_r, int n_phi, double r_min, double r_max, int plus,
                        const double *self, const double *sigma, const int64_t *dest,
                        int64_t n_dest, double *f_r, double *f_phi)
{
    return or_forward_particle_o(n_r, n_phi, r_min, r_max, plus, 2, self, sigma, dest, n_dest,
                                 f_r, f_phi);
}

/* ------------------------------------------------------------------------ */
/* Two patches of one log-polar grid (Sec. 3.2.1, Eq. 27-29 with the         */
/* interaction and origin terms).  Rows of the common grid are indexed by    */
/* any integer k: row k spans [r_min beta^k, r_min beta^(k+1)], centre       */
/* r_min beta^k (1 + beta)/2, with beta and dphi from the destination patch  */
/* (N_dst rows from r_min to r_max).  The source patch holds rows            */
/* s0 ... s0 + N_src - 1.  Destination row i and source row i' are at the    */
/* offset m = i - (s0 + i'); tables are stored by m' = i - i' in              */
/* [-(N_src-1), N_dst-1], row m' + N_src - 1, each entry the kernel of        */
/* offset m = m' - s0.  Source slopes are taken inside the source patch      */
/* (one-sided on its first and last rows).                                    */
/*                                                                          */
/* Origin wedges (the cells R^hat_j = [0, r_w] x [phi_j' +- dphi/2] below    */
/* the source patch, r_w = r_min beta^s0; the paper uses barred kernels for  */
/* them without defining them).  Reading: the same integrands as Eq. 30-32   */
/* and A22-A24 over the wedge, the wedge's radial centre taken as r_w / 2    */
/* (the arithmetic centre, as for every other cell), its density value at    */
/* that centre, its azimuthal slope by periodic central differences and its  */
/* radial slope by the one-sided difference towards the first source row.   */
/* In units of r_i (eta = rbar / r_i, xi = phibar - phi_j, xi_c = -n dphi):  */
/*   Tw_r0 = -int eta (1 - eta cos xi) / F^3,                               */
/*   Tw_rr = -int eta (1 - eta cos xi) (eta - eta_c) / F^3,                 */
/*   Tw_rphi = -int eta (1 - eta cos xi) (xi - xi_c) / F^3,                 */
/*   Tw_phi0 = int eta^2 sin xi / F^3, and likewise Tw_phir, Tw_phiphi,      */
/* over eta in [0, r_w / r_i], eta_c = r_w / (2 r_i), xi in [xi_c +- dphi/2]; */
/* F^r += sigma Tw_r0 + r_i delta^r Tw_rr + delta^phi Tw_rphi, and the same  */
/* for F^phi.  The integrand is smooth (the wedge lies inside r_min), so a    */
/* 24-point Gauss-Legendre rule in xi and adaptive Gauss-Legendre in eta are */
/* used.  For the particle methods a wedge is the point mass                 */
/* sigma r_w^2 dphi / 2 (its exact area) at (r_w / 2, phi_j').               */
/* ------------------------------------------------------------------------ */
int or_patch_tables(int n_src, int s0, int n_dst, int n_phi, double r_min, double r_max,
                    int n_tpz, int table_mode, const double *self, double *T)
{
    double beta, dphi;
    if (or_geometry(n_dst, n_phi, r_min, r_max, NULL, NULL, &beta, &dphi)) return -1;
    if (n_src < 2 || (table_mode == 0 && n_tpz < 1) || table_mode < 0 || table_mode > 1 ||
        (n_phi % 2) != 0)
        return -1;
    gl_init();
    const long rows = (long)n_src + n_dst - 1;
    const long plane = rows * (long)n_phi;
    static const double par[6] = {1, 1, -1, -1, -1, 1};
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
#endif
    for (long row = 0; row < rows; ++row)
        for (int nrep = 0; nrep <= n_phi / 2; ++nrep) {
            const int m = (int)(row - (n_src - 1)) - s0;
            double t[6];
            table_entry(beta, dphi, n_tpz, table_mode, m, nrep, self, t);
            long cpos = nrep, cneg = (n_phi - nrep) % n_phi;
            for (int k = 0; k < 6; ++k) {
                T[k * plane + row * n_phi + cpos] = t[k];
                if (cneg != cpos) T[k * plane + row * n_phi + cneg] = par[k] * t[k];
            }
        }
    return 0;
}

typedef struct { double xic, dphi, eta_c; } wedge_ctx;

static void wedge_integrand(double eta, void *vctx, double *out)
{
    const wedge_ctx *c = (const wedge_ctx *)vctx;
    const int n = 24;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < n; ++k) {
        const double xi = c->xic + 0.5 * c->dphi * gl_x[n][k];
        const double w = 0.5 * c->dphi * gl_w[n][k];
        const double F = Fpol(eta, sin(0.5 * xi));
        const double iF3 = 1.0 / (F * F * F);
        const double fr = eta * (1.0 - eta * cos(xi)) * iF3;
        const double fp = eta * eta * sin(xi) * iF3;
        const double dx = xi - c->xic;
        a[0] += w * fr;
        a[1] += w * fr * (eta - c->eta_c);
        a[2] += w * fr * dx;
        a[3] += w * fp;
        a[4] += w * fp * (eta - c->eta_c);
        a[5] += w * fp * dx;
    }
    for (int k = 0; k < 6; ++k) out[k] = a[k];
}

/* Wedge tables [6][N_dst][N_phi] (order r0, rr, rphi, phi0, phir, phiphi);
 * column n = (j - j') mod N_phi.  method 0: the integrals above; 1: point
 * masses. */
int or_wedge_tables(int n_dst, int n_phi, double r_min, double r_max, int s0, int method,
                    double *T)
{
    double beta, dphi;
    double *rc = (double *)malloc(sizeof(double) * n_dst);
    if (!rc) return -2;
    if (or_geometry(n_dst, n_phi, r_min, r_max, rc, NULL, &beta, &dphi) || s0 > 0 ||
        method < 0 || method > 1) {
        free(rc);
        return -1;
    }
    gl_init();
    const double r_w = r_min * pow(beta, s0);
    const long plane = (long)n_dst * n_phi;
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
#endif
    for (int i = 0; i < n_dst; ++i)
        for (int n = 0; n < n_phi; ++n) {
            const int nrep = n <= n_phi / 2 ? n : n - n_phi;
            const double xic = -nrep * dphi;
            const double eta_w = r_w / rc[i];
            double t[6];
            if (method == 0) {
                wedge_ctx c = {xic, dphi, 0.5 * eta_w};
                adapt_gl(wedge_integrand, &c, 6, 0.0, eta_w, 1e-14, t);
                t[0] = -t[0];
                t[1] = -t[1];
                t[2] = -t[2];
            } else {
                const double ec = 0.5 * eta_w, A = 0.5 * eta_w * eta_w * dphi;
                const double F = Fpol(ec, sin(0.5 * xic));
                const double iF3 = 1.0 / (F * F * F);
                t[0] = A * (ec * cos(xic) - 1.0) * iF3;
                t[3] = A * ec * sin(xic) * iF3;
                t[1] = t[2] = t[4] = t[5] = 0.0;
            }
            for (int k = 0; k < 6; ++k) T[k * plane + (long)i * n_phi + n] = t[k];
        }
    free(rc);
    return 0;
}

/* Forces on the destination patch from the source patch (tables T of
 * or_patch_tables) and, when Tw and sigma_w are given, from the origin
 * wedges (tables Tw of or_wedge_tables, wedge densities sigma_w[N_phi]).
 * c0: the source patch and its wedges turned by c0 whole cells in phi
 * (source column j' centred at (j' + c0 + 1/2) dphi): the tables are taken
 * at the offset j - j' - c0 (mod N_phi). */
static int wrap_n(long n, int n_phi)
{
    n %= n_phi;
    return (int)(n < 0 ? n + n_phi : n);
}

int or_patch_forward(int n_src, int s0, int c0, int n_dst, int n_phi, double r_min, double r_max,
                     const double *T, const double *sigma_src, const double *Tw,
                     const double *sigma_w, const int64_t *dest, int64_t n_dest, double *f_r,
                     double *f_phi)
{
    double beta, dphi;
    double *rd = (double *)malloc(sizeof(double) * n_dst);
    double *rs = (double *)malloc(sizeof(double) * n_src);
    const long Ns = (long)n_src * n_phi;
    double *dr = (double *)malloc(sizeof(double) * Ns);
    double *dp = (double *)malloc(sizeof(double) * Ns);
    double *wr = (double *)malloc(sizeof(double) * n_phi);
    double *wp = (double *)malloc(sizeof(double) * n_phi);
    int rcode = 0;
    if (!rd || !rs || !dr || !dp || !wr || !wp) { rcode = -2; goto done; }
    if (or_geometry(n_dst, n_phi, r_min, r_max, rd, NULL, &beta, &dphi) || n_src < 2) {
        rcode = -1;
        goto done;
    }
    for (int k = 0; k < n_src; ++k) rs[k] = r_min * pow(beta, s0 + k) * 0.5 * (1.0 + beta);
    or_channels(n_src, n_phi, rs, dphi, sigma_src, dr, dp);
    if (Tw && sigma_w) {
        const double r_w = r_min * pow(beta, s0), rh = 0.5 * r_w;
        for (int j = 0; j < n_phi; ++j) {
            wp[j] = (sigma_w[(j + 1) % n_phi] - sigma_w[(j + n_phi - 1) % n_phi]) / (2.0 * dphi);
            wr[j] = (sigma_src[j] - sigma_w[j]) / (rs[0] - rh);
        }
    }
    {
        const long rows = (long)n_src + n_dst - 1;
        const long plane = rows * (long)n_phi, wplane = (long)n_dst * n_phi;
        const long nd = dest ? (long)n_dest : (long)n_dst * n_phi;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (long q = 0; q < nd; ++q) {
            const long cell = dest ? (long)dest[q] : q;
            const int i = (int)(cell / n_phi), j = (int)(cell % n_phi);
            acc_t a0 = {0, 0}, ar = {0, 0}, ap = {0, 0}, b0 = {0, 0}, br = {0, 0}, bp = {0, 0};
            for (int ip = 0; ip < n_src; ++ip) {
                const long row = (long)(i - ip) + (n_src - 1);
                const double *sg = sigma_src + (long)ip * n_phi, *gr = dr + (long)ip * n_phi,
                             *gp = dp + (long)ip * n_phi;
                double x0 = 0, xr = 0, xp = 0, y0 = 0, yr = 0, yp = 0;
                for (int jp = 0; jp < n_phi; ++jp) {
                    const long t = row * n_phi + wrap_n((long)j - jp - c0, n_phi);
                    x0 += sg[jp] * T[t];
                    xr += gr[jp] * T[plane + t];
                    xp += gp[jp] * T[2 * plane + t];
                    y0 += sg[jp] * T[3 * plane + t];
                    yr += gr[jp] * T[4 * plane + t];
                    yp += gp[jp] * T[5 * plane + t];
                }
                acc_add(&a0, x0); acc_add(&ar, xr); acc_add(&ap, xp);
                acc_add(&b0, y0); acc_add(&br, yr); acc_add(&bp, yp);
            }
            if (Tw && sigma_w) {
                double x0 = 0, xr = 0, xp = 0, y0 = 0, yr = 0, yp = 0;
                for (int jp = 0; jp < n_phi; ++jp) {
                    const long t = (long)i * n_phi + wrap_n((long)j - jp - c0, n_phi);
                    x0 += sigma_w[jp] * Tw[t];
                    xr += wr[jp] * Tw[wplane + t];
                    xp += wp[jp] * Tw[2 * wplane + t];
                    y0 += sigma_w[jp] * Tw[3 * wplane + t];
                    yr += wr[jp] * Tw[4 * wplane + t];
                    yp += wp[jp] * Tw[5 * wplane + t];
                }
                acc_add(&a0, x0); acc_add(&ar, xr); acc_add(&ap, xp);
                acc_add(&b0, y0); acc_add(&br, yr); acc_add(&bp, yp);
            }
            f_r[q] = acc_get(&a0) + rd[i] * acc_get(&ar) + acc_get(&ap);
            f_phi[q] = acc_get(&b0) + rd[i] * acc_get(&br) + acc_get(&bp);
        }
    }
done:
    free(rd); free(rs); free(dr); free(dp); free(wr); free(wp);
    return rcode;
}

/* Transpose of or_patch_forward, as a plain double sum at chosen source
 * cells: g[p] = sum over destination cells q of
 * v_r[q] dF_r[q]/dsigma_src[p] + v_phi[q] dF_phi[q]/dsigma_src[p], with the
 * slopes taken inside the source patch (order 2, as the forward).
 * v_r, v_phi: [n_dst][n_phi]; src: flat source indices (NULL = all).
 * With the wedge tables Tw (NULL: no wedges) also gw[n_phi], the gradient
 * with respect to the wedge densities (all of them), and the wedges' radial
 * slope -- the difference towards the first source row -- adds to the
 * gradient of that row (to g only where src is NULL, i.e. the full grid). */
static void adj_u_patch(int n_src, int n_dst, int n_phi, const double *rd, const double *T,
                        const double *v_r, const double *v_p, int ip, int jp, int c0,
                        double *us, double *ug, double *uh)
{
    const long rows = (long)n_src + n_dst - 1;
    const long plane = rows * (long)n_phi;
    acc_t s = {0, 0}, g = {0, 0}, h = {0, 0};
    for (int i = 0; i < n_dst; ++i) {
        const long row = (long)(i - ip) + (n_src - 1);
        const double *t0 = T + row * n_phi, *tr = T + plane + row * n_phi,
                     *tp = T + 2 * plane + row * n_phi;
        const double *u0 = T + 3 * plane + row * n_phi, *ur = T + 4 * plane + row * n_phi,
                     *up = T + 5 * plane + row * n_phi;
        const double *vr = v_r + (long)i * n_phi, *vp = v_p + (long)i * n_phi;
        double xs = 0, xg = 0, xh = 0;
        for (int j = 0; j < n_phi; ++j) {
            const int n = wrap_n((long)j - jp - c0, n_phi);
            xs += vr[j] * t0[n] + vp[j] * u0[n];
            xg += vr[j] * tr[n] + vp[j] * ur[n];
            xh += vr[j] * tp[n] + vp[j] * up[n];
        }
        acc_add(&s, xs);
        acc_add(&g, rd[i] * xg);
        acc_add(&h, xh);
    }
    *us = acc_get(&s);
    *ug = acc_get(&g);
    *uh = acc_get(&h);
}

/* sums of the cotangents against the wedge tables for wedge jp */
static void adj_u_wedge(int n_dst, int n_phi, const double *rd, const double *Tw,
                        const double *v_r, const double *v_p, int jp, int c0, double *us,
                        double *ug, double *uh)
{
    const long wplane = (long)n_dst * n_phi;
    acc_t s = {0, 0}, g = {0, 0}, h = {0, 0};
    for (int i = 0; i < n_dst; ++i) {
        const double *vr = v_r + (long)i * n_phi, *vp = v_p + (long)i * n_phi;
        double xs = 0, xg = 0, xh = 0;
        for (int j = 0; j < n_phi; ++j) {
            const long t = (long)i * n_phi + wrap_n((long)j - jp - c0, n_phi);
            xs += vr[j] * Tw[t] + vp[j] * Tw[3 * wplane + t];
            xg += vr[j] * Tw[wplane + t] + vp[j] * Tw[4 * wplane + t];
            xh += vr[j] * Tw[2 * wplane + t] + vp[j] * Tw[5 * wplane + t];
        }
        acc_add(&s, xs);
        acc_add(&g, rd[i] * xg);
        acc_add(&h, xh);
    }
    *us = acc_get(&s);
    *ug = acc_get(&g);
    *uh = acc_get(&h);
}

int or_patch_adjoint(int n_src, int s0, int c0, int n_dst, int n_phi, double r_min, double r_max,
                     const double *T, const double *v_r, const double *v_phi,
                     const int64_t *src, int64_t n_idx, double *g, const double *Tw,
                     double *gw)
{
    double beta, dphi;
    double *rd = (double *)malloc(sizeof(double) * n_dst);
    double *rs = (double *)malloc(sizeof(double) * n_src);
    int rcode = 0;
    if (!rd || !rs) { rcode = -2; goto done; }
    if (or_geometry(n_dst, n_phi, r_min, r_max, rd, NULL, &beta, &dphi) || n_src < 2 ||
        n_phi < 3) {
        rcode = -1;
        goto done;
    }
    for (int k = 0; k < n_src; ++k) rs[k] = r_min * pow(beta, s0 + k) * 0.5 * (1.0 + beta);
    {
        const long N = (long)n_src * n_phi;
        const long ns = src ? (long)n_idx : N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (long q = 0; q < ns; ++q) {
            const long p = src ? (long)src[q] : q;
            const int ip = (int)(p / n_phi), jp = (int)(p % n_phi);
            double us, ug, uh, a, b, c;
            adj_u_patch(n_src, n_dst, n_phi, rd, T, v_r, v_phi, ip, jp, c0, &us, &ug, &uh);
            double tot = us;
            for (int i2 = ip - 1; i2 <= ip + 1; ++i2) {
                if (i2 < 0 || i2 >= n_src) continue;
                const double cf = dr_coef(n_src, rs, 2, i2, ip);
                if (cf == 0.0) continue;
                adj_u_patch(n_src, n_dst, n_phi, rd, T, v_r, v_phi, i2, jp, c0, &a, &b, &c);
                tot += cf * b;
            }
            for (int d = -1; d <= 1; d += 2) {
                const int j2 = ((jp - d) % n_phi + n_phi) % n_phi;
                adj_u_patch(n_src, n_dst, n_phi, rd, T, v_r, v_phi, ip, j2, c0, &a, &b, &c);
                tot += dp_coef(2, dphi, d) * c;
            }
            g[q] = tot;
        }
    }
    if (Tw && gw) {
        const double rh = 0.5 * r_min * pow(beta, s0), inv = 1.0 / (rs[0] - rh);
        double *ug0 = (double *)malloc(sizeof(double) * n_phi);
        double *us0 = (double *)malloc(sizeof(double) * n_phi);
        double *uh0 = (double *)malloc(sizeof(double) * n_phi);
        if (!ug0 || !us0 || !uh0) { free(ug0); free(us0); free(uh0); rcode = -2; goto done; }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (int jp = 0; jp < n_phi; ++jp)
            adj_u_wedge(n_dst, n_phi, rd, Tw, v_r, v_phi, jp, c0, &us0[jp], &ug0[jp], &uh0[jp]);
        for (int jp = 0; jp < n_phi; ++jp) {
            /* sigma_w[jp] enters the wedge density, its radial slope
             * (sigma_src[0] - sigma_w) / (r_0 - r_w / 2) and its periodic
             * azimuthal slope */
            double tot = us0[jp] - inv * ug0[jp];
            for (int d = -1; d <= 1; d += 2)
                tot += dp_coef(2, dphi, d) * uh0[((jp - d) % n_phi + n_phi) % n_phi];
            gw[jp] = tot;
            if (!src) g[jp] += inv * ug0[jp];   /* the first source row */
        }
        free(ug0); free(us0); free(uh0);
    }
done:
    free(rd); free(rs);
    return rcode;
}

/* Particle and modified particle methods between patches, in physical
 * coordinates: source cells are point masses sigma r dr dphi at their
 * centres, wedges (if sigma_w) point masses sigma r_w^2 dphi / 2 at
 * (r_w / 2, phi_j'); a destination cell that coincides with a source cell
 * feels no force from it, and plus = 1 adds there the self-cell correction
 * of Eq. 34-37 with the source patch's slopes.  c0: the source patch and
 * its wedges turned by c0 whole cells (source column j' at azimuth
 * (j' + c0 + 1/2) dphi). */
int or_patch_particle(int n_src, int s0, int c0, int n_dst, int n_phi, double r_min, double r_max,
                      int plus, const double *self, const double *sigma_src,
                      const double *sigma_w, const int64_t *dest, int64_t n_dest, double *f_r,
                      double *f_phi)
{
    double beta, dphi;
    double *rd = (double *)malloc(sizeof(double) * n_dst);
    double *rs = (double *)malloc(sizeof(double) * n_src);
    const long Ns = (long)n_src * n_phi;
    double *dr = (double *)malloc(sizeof(double) * Ns);
    double *dp = (double *)malloc(sizeof(double) * Ns);
    int rcode = 0;
    if (!rd || !rs || !dr || !dp) { rcode = -2; goto done; }
    if (or_geometry(n_dst, n_phi, r_min, r_max, rd, NULL, &beta, &dphi) || n_src < 2) {
        rcode = -1;
        goto done;
    }
    for (int k = 0; k < n_src; ++k) rs[k] = r_min * pow(beta, s0 + k) * 0.5 * (1.0 + beta);
    or_channels(n_src, n_phi, rs, dphi, sigma_src, dr, dp);
    {
        const double r_w = r_min * pow(beta, s0);
        const long nd = dest ? (long)n_dest : (long)n_dst * n_phi;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (long q = 0; q < nd; ++q) {
            const long cell = dest ? (long)dest[q] : q;
            const int i = (int)(cell / n_phi), j = (int)(cell % n_phi);
            const double ri = rd[i];
            acc_t ar = {0, 0}, ap = {0, 0};
            for (int ip = 0; ip < n_src; ++ip) {
                const int k = s0 + ip;
                const double r2 = rs[ip];
                const double area = 0.5 * (pow(beta, 2.0 * (k + 1)) - pow(beta, 2.0 * k)) *
                                    r_min * r_min * dphi;
                for (int jp = 0; jp < n_phi; ++jp) {
                    if (k == i && wrap_n((long)jp + c0 - j, n_phi) == 0) continue;
                    const double M = sigma_src[(long)ip * n_phi + jp] * area;
                    if (M == 0.0) continue;
                    const double d = ((long)jp + c0 - j) * dphi;
                    const double sh = sin(0.5 * d);
                    const double D = (ri - r2) * (ri - r2) + 4.0 * ri * r2 * sh * sh;
                    const double w = M / (D * sqrt(D));
                    acc_add(&ar, w * (r2 * cos(d) - ri));
                    acc_add(&ap, w * r2 * sin(d));
                }
            }
            if (sigma_w) {
                const double r2 = 0.5 * r_w, area = 0.5 * r_w * r_w * dphi;
                for (int jp = 0; jp < n_phi; ++jp) {
                    const double M = sigma_w[jp] * area;
                    if (M == 0.0) continue;
                    const double d = ((long)jp + c0 - j) * dphi;
                    const double sh = sin(0.5 * d);
                    const double D = (ri - r2) * (ri - r2) + 4.0 * ri * r2 * sh * sh;
                    const double w = M / (D * sqrt(D));
                    acc_add(&ar, w * (r2 * cos(d) - ri));
                    acc_add(&ap, w * r2 * sin(d));
                }
            }
            double fr = acc_get(&ar), fp = acc_get(&ap);
            const int ip = i - s0;
            if (plus && ip >= 0 && ip < n_src) {
                const long c = (long)ip * n_phi + wrap_n((long)j - c0, n_phi);
                fr += sigma_src[c] * self[0] + ri * dr[c] * self[1];
                fp += dp[c] * self[2];
            }
            f_r[q] = fr;
            f_phi[q] = fp;
        }
    }
done:
    free(rd); free(rs); free(dr); free(dp);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Cartesian coordinates (Sec. 3.1, Eq. 6-21, A1-A16).  An N_x x N_y grid of */
/* cells Delta x by Delta y; cell (i, j), 0-based, i along x and j along y.  */
/* Arrays are row-major [N_x][N_y].  Tables are indexed by the offsets        */
/* m = i - i', n = j - j' (destination minus source), stored at             */
/* [k][m + N_x - 1][n + N_y - 1], kernels in the order                       */
/*   K^{x,0}, K^{x,x}, K^{x,y}, K^{y,0}, K^{y,y}, K^{y,x}                   */
/* (Eq. 13-15 and A5-A7).  The source centre relative to the destination is */
/* (X, Y) = (-m Delta x, -n Delta y).                                        */
/*                                                                          */
/* Second-order tables: the closed forms A8-A13 (cart_closed above) for     */
/* cells within three cell sizes of the destination; beyond that the same   */
/* integrals by a tensor Gauss-Legendre rule, whose order per direction is  */
/* chosen so that (h / 2d)^(2n) < 1e-17 (the closed double differences lose */
/* digits to cancellation far away).                                        */
/* ------------------------------------------------------------------------ */
static void cart_gl(double X, double Y, double dx, double dy, int nx, int ny, double K[6])
{
    const double *xg = gl_x[nx], *wx = gl_w[nx], *yg = gl_x[ny], *wy = gl_w[ny];
    acc_t a[6];
    for (int k = 0; k < 6; ++k) a[k].s = a[k].c = 0;
    for (int p = 0; p < nx; ++p) {
        const double u = 0.5 * dx * xg[p];            /* xbar - x_i' */
        const double x = X + u;                        /* xbar - x_i  */
        for (int q = 0; q < ny; ++q) {
            const double v = 0.5 * dy * yg[q];        /* ybar - y_j' */
            const double y = Y + v;                    /* ybar - y_j  */
            const double r2 = x * x + y * y;
            const double w = 0.25 * dx * dy * wx[p] * wy[q] / (r2 * sqrt(r2));
            acc_add(&a[0], w * x);
            acc_add(&a[1], w * x * u);
            acc_add(&a[2], w * x * v);
            acc_add(&a[3], w * y);
            acc_add(&a[4], w * y * v);
            acc_add(&a[5], w * y * u);
        }
    }
    for (int k = 0; k < 6; ++k) K[k] = acc_get(&a[k]);
}

static int gl_order_for(double q)
{
    static const int ns[7] = {2, 3, 4, 6, 8, 12, 16};
    for (int k = 0; k < 7; ++k)
        if (pow(q, 2 * ns[k]) < 1e-17) return ns[k];
    return 16;
}

/* method: 0 second order (Eq. 10-15), 1 particle (Eq. 20 kernel, no
 * correction), 2 modified particle (Eq. 20 plus the self-cell correction
 * of Eq. 21, i.e. K^{x,x}_{00} and K^{y,y}_{00} in the (0, 0) entries; the
 * other self terms vanish by symmetry).  Particle masses sigma Dx Dy. */
int or_cart_tables(int n_x, int n_y, double dx, double dy, int method, double *T)
{
    if (n_x < 2 || n_y < 2 || !(dx > 0) || !(dy > 0) || method < 0 || method > 2) return -1;
    gl_init();
    const long rows = 2L * n_x - 1, cols = 2L * n_y - 1, plane = rows * cols;
    const double hmax = dx > dy ? dx : dy;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long row = 0; row < rows; ++row) {
        const int m = (int)row - (n_x - 1);
        for (long col = 0; col < cols; ++col) {
            const int n = (int)col - (n_y - 1);
            const double X = -m * dx, Y = -n * dy;
            const double d = sqrt(X * X + Y * Y);
            double K[6] = {0, 0, 0, 0, 0, 0};
            if (method == 0) {
                if (d < 3.0 * hmax)
                    cart_closed(X - 0.5 * dx, X + 0.5 * dx, Y - 0.5 * dy, Y + 0.5 * dy, X, Y, K);
                else
                    cart_gl(X, Y, dx, dy, gl_order_for(0.5 * dx / d), gl_order_for(0.5 * dy / d), K);
            } else if (m != 0 || n != 0) {
                const double w = dx * dy / (d * d * d);
                K[0] = w * X;
                K[3] = w * Y;
            } else if (method == 2) {
                double S[6];
                cart_closed(-0.5 * dx, 0.5 * dx, -0.5 * dy, 0.5 * dy, 0.0, 0.0, S);
                K[1] = S[1];
                K[4] = S[4];
            }
            for (int k = 0; k < 6; ++k) T[k * plane + row * cols + col] = K[k];
        }
    }
    return 0;
}

/* Cell slopes: central differences, one-sided two-point differences on the
 * first and last cells of each direction. */
static void cart_slopes(int n_x, int n_y, double dx, double dy, const double *s, double *gx,
                        double *gy)
{
    for (int i = 0; i < n_x; ++i)
        for (int j = 0; j < n_y; ++j) {
            const long c = (long)i * n_y + j;
            if (i == 0) gx[c] = (s[c + n_y] - s[c]) / dx;
            else if (i == n_x - 1) gx[c] = (s[c] - s[c - n_y]) / dx;
            else gx[c] = (s[c + n_y] - s[c - n_y]) / (2.0 * dx);
            if (j == 0) gy[c] = (s[c + 1] - s[c]) / dy;
            else if (j == n_y - 1) gy[c] = (s[c] - s[c - 1]) / dy;
            else gy[c] = (s[c + 1] - s[c - 1]) / (2.0 * dy);
        }
}

int or_cart_slopes(int n_x, int n_y, double dx, double dy, const double *sigma, double *gx,
                   double *gy)
{
    if (n_x < 2 || n_y < 2) return -1;
    cart_slopes(n_x, n_y, dx, dy, sigma, gx, gy);
    return 0;
}

/* F^x, F^y as the plain double sums of Eq. 9-12 and A1-A4 at the chosen
 * destinations (flat i * N_y + j), or at every cell. */
int or_cart_forward(int n_x, int n_y, double dx, double dy, const double *T, const double *sigma,
                    const int64_t *dest, int64_t n_dest, double *f_x, double *f_y)
{
    if (n_x < 2 || n_y < 2) return -1;
    const long N = (long)n_x * n_y;
    const long cols = 2L * n_y - 1, plane = (2L * n_x - 1) * cols;
    double *gx = (double *)malloc(sizeof(double) * N), *gy = (double *)malloc(sizeof(double) * N);
    if (!gx || !gy) { free(gx); free(gy); return -2; }
    cart_slopes(n_x, n_y, dx, dy, sigma, gx, gy);
    const long nd = dest ? (long)n_dest : N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long q = 0; q < nd; ++q) {
        const long cell = dest ? (long)dest[q] : q;
        const int i = (int)(cell / n_y), j = (int)(cell % n_y);
        acc_t ax = {0, 0}, ay = {0, 0};
        for (int ip = 0; ip < n_x; ++ip) {
            const long row = (long)(i - ip) + (n_x - 1);
            const long base = row * cols + (j + n_y - 1);   /* column of jp = 0 */
            double sx = 0, sy = 0;
            for (int jp = 0; jp < n_y; ++jp) {
                const long t = base - jp;
                const long c = (long)ip * n_y + jp;
                sx += sigma[c] * T[t] + gx[c] * T[plane + t] + gy[c] * T[2 * plane + t];
                sy += sigma[c] * T[3 * plane + t] + gy[c] * T[4 * plane + t] +
                      gx[c] * T[5 * plane + t];
            }
            acc_add(&ax, sx);
            acc_add(&ay, sy);
        }
        f_x[q] = acc_get(&ax);
        f_y[q] = acc_get(&ay);
    }
    free(gx); free(gy);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
