// pf_tables.hip -- one-time FP64 construction of the force-kernel tables and
// their spectra (Sec. 3.2.1 and 4; Eq. 30-33, 41-46, A22-A24).
//
// Kernel tables.  For destination-minus-source offset (m, n) the six kernels
// are integrals over the source cell in eta = rbar / r_i and
// xi = phibar - phi_j (Eq. 33):
//   eta in [2 beta^-m / (1+beta), 2 beta^(1-m) / (1+beta)],
//   xi  in [xi_c - dphi/2, xi_c + dphi/2],  xi_c = -n dphi  (n wrapped to
//   (-n_phi/2, n_phi/2]),  F = sqrt(eta^2 - 2 eta cos xi + 1),
//   K^{r,0}  = -int int eta (1 - eta cos xi) / F^3
//   K^{r,r}  = -int int eta (1 - eta cos xi) (eta - beta^-m) / F^3
//   K^{r,phi}= -int int eta (1 - eta cos xi) (xi - xi_c) / F^3
//   K^{phi,0}=  int int eta^2 sin xi / F^3
//   K^{phi,r}=  int int eta^2 sin xi (eta - beta^-m) / F^3
//   K^{phi,phi}=int int eta^2 sin xi (xi - xi_c) / F^3.
// SIM (Sec. 4): K^{r,0}, K^{r,r}, K^{r,phi}, K^{phi,phi} take the composite
// trapezoid rule with n_tpz panels in xi (Eq. 41-43) of the exact eta
// integral; K^{phi,0} and K^{phi,r} are exact (A30-A31).  The exact table
// mode takes those four xi integrals converged as well (graded Gauss-
// Legendre panels towards the singularities in xi).  Here every exact
// one-dimensional integral is evaluated by 16-point Gauss-Legendre on panels
// graded geometrically towards the nearest complex singularity of the
// integrand (eta = exp(+-i xi)), which keeps each panel's Bernstein-ellipse
// ratio above 3.7 and so the rule exact to rounding.  The xi integral of the
// K^{phi,.} kernels is done in closed form first:
//   int eta^2 sin xi / F^3 dxi = -eta / F,
//   1/F(xi_l) - 1/F(xi_u) = 4 eta sin(xi_c) sin(dphi/2) / (F_l F_u (F_l + F_u)).
//
// Self cell (m = n = 0, Sec. 4, Eq. 44-46, Fig. 1): the fan-shaped cell of
// centre (1, 0) (the kernels depend only on beta and dphi, Eq. 33) is
// covered by a Cartesian grid of cells of size Delta x / per by
// Delta y / per, aligned so (1, 0) is a cell centre, a cell kept iff its
// centre lies in the closed fan.  The Cartesian second-order method
// (Eq. 9-15, closed forms A8-A13) gives the force at (1, 0) of the test
// densities 1, rbar - 1 and phibar, with the densities' slopes taken at each
// Cartesian centre; these are K^{r,0}_{00}, K^{r,r}_{00} and
// K^{phi,phi}_{00}.  The other three self kernels vanish by symmetry.  The
// exact self mode takes the same three constants as the exact integrals over
// the fan (principal value for K^{r,0}, k_selfpv).
//
// Spectra.  With T_rr and T_phir multiplied by beta^m (the r_i / r_i'
// factor of Eq. 28), all six tables are 2-D transformed (rows along phi,
// then columns along u, padded to L), the azimuthal slope kernels folded in
// with the periodic central difference, the radial slope's circular central
// difference D(k) = 2i ca sin(2 pi k / L) folded in, and normalised by
// 1/(L n_phi):
//   E'_r = F(T_r0) + i sin(2 pi k / n_phi) / dphi * F(T_rphi) + D Q_r
//   Q_r  = F(beta^m T_rr)
//   E'_p = F(T_p0) + i sin(2 pi k / n_phi) / dphi * F(T_pphi) + D Q_p
//   Q_p  = F(beta^m T_pr)
// (with slope order 4 the five-point differences' symbols take the place
// of the sines, k_fold) stored for k_u in [0, L/2] only, as pairs (E', Q)
// (k_fold).  E_p and Q_p
// vanish at the azimuthal bins 0 and n_phi/2 (odd kernels) and are not
// stored there.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "pf_common.hpp"

namespace pf {

// 8- and 16-point Gauss-Legendre rules on [-1, 1] (positive half).
__constant__ double kGL8x[4] = {0.18343464249564978, 0.52553240991632899, 0.79666647741362673,
                                0.96028985649753618};
__constant__ double kGL8w[4] = {0.36268378337836177, 0.31370664587788705, 0.22238103445337434,
                                0.10122853629037669};
__constant__ double kGL16x[8] = {0.095012509837637454, 0.28160355077925892, 0.45801677765722737,
                                 0.61787624440264377,  0.755404408355003,   0.86563120238783176,
                                 0.9445750230732326,   0.98940093499164994};
__constant__ double kGL16w[8] = {0.18945061045506859,  0.18260341504492361,  0.16915651939500262,
                                 0.14959598881657676,  0.12462897125553403,  0.095158511682492591,
                                 0.062253523938647706, 0.027152459411754037};

__device__ __forceinline__ double Fpol(double eta, double sh) {
    const double d = eta - 1.0;
    return sqrt(d * d + 4.0 * eta * sh * sh);
}

// 16-point Gauss-Legendre over panels of [a, b] graded towards the complex
// point (pr, pi).  f(eta, weight) accumulates.
template <class Fn>
__device__ void graded_gl16(double a, double b, double pr, double pim, Fn &f) {
    auto panel = [&](double lo, double hi) {
        const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double dx = h * kGL16x[k], w = h * kGL16w[k];
            f(c - dx, w);
            f(c + dx, w);
        }
    };
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    if (hypot(c - pr, pim) >= 2.0 * h) {
        panel(a, b);
        return;
    }
    const double q = fmin(fmax(pr, a), b);
    double w0 = fmax(pim, fabs(pr - q));
    if (!(w0 > 0)) w0 = 1e-12 * (b - a);
    // right of q
    {
        const double len = b - q;
        double lo = 0.0, w = w0;
        while (lo < len) {
            const double hi = fmin(lo + w, len);
            panel(q + lo, q + hi);
            lo = hi;
            w *= 2.0;
        }
    }
    // left of q
    {
        const double len = q - a;
        double lo = 0.0, w = w0;
        while (lo < len) {
            const double hi = fmin(lo + w, len);
            panel(q - hi, q - lo);
            lo = hi;
            w *= 2.0;
        }
    }
}

struct TabGeo {
    double beta, dphi, lnb;
    int n_r, n_phi, L, n_tpz;
    int exact;    // 1: azimuthal integrals converged instead of n_tpz trapezoids
    int method;   // PF_METHOD_*
    int n_in, s0; // source rows s0 .. s0 + n_in - 1 (n_r destination rows)
};

// Particle methods (Eq. 35-37, 56-62).  A source cell is the point mass
// Mbar = sigma r_i' dr_i' dphi at its centre; with r_i' = rho r_i,
// rho = beta^-m, dr / r = 2 (beta - 1)/(beta + 1) for arithmetic centres and
// xi_c = -n dphi its force on the destination centre, per unit sigma, is
//   F_r   = rho^2 c_A dphi (rho cos xi_c - 1) / F^3,
//   F_phi = rho^3 c_A dphi sin xi_c / F^3,  F^2 = (1 - rho)^2 + 4 rho sin^2(xi_c/2),
// independent of r_i (Eq. 33).  No self force; the modified method puts the
// self-cell correction in the (0, 0) entries of K^{r,0}, K^{r,r}, K^{phi,phi}.
__device__ void particle_entry(const TabGeo &g, int m, int nrep, const double *selfk,
                               double *t) {
    for (int k = 0; k < 6; ++k) t[k] = 0.0;
    if (m == 0 && nrep == 0) {
        if (g.method == PF_METHOD_PARTICLE_PLUS) {
            t[0] = selfk[0];
            t[1] = selfk[1];
            t[5] = selfk[2];
        }
        return;
    }
    const double rho = exp(-m * g.lnb);
    const double xic = -nrep * g.dphi;
    const double cA = 2.0 * (g.beta - 1.0) / (g.beta + 1.0);
    const double sh = sin(0.5 * xic);
    const double D = (1.0 - rho) * (1.0 - rho) + 4.0 * rho * sh * sh;
    const double w = rho * rho * cA * g.dphi / (D * sqrt(D));
    double s, c;
    sincos(xic, &s, &c);
    t[0] = w * (rho * c - 1.0);
    t[3] = w * rho * s;
}

// All six kernels of offset (m, n_rep) into t[6]:
// r0, rr, rphi, phi0, phir, phiphi (unscaled by beta^m).
__device__ void table_entry(const TabGeo &g, int m, int nrep, const double *selfk, double *t) {
    if (m == 0 && nrep == 0) {
        t[0] = selfk[0];
        t[1] = selfk[1];
        t[2] = 0.0;
        t[3] = 0.0;
        t[4] = 0.0;
        t[5] = selfk[2];
        return;
    }
    const double rho = exp(-m * g.lnb);
    const double el = 2.0 * rho / (1.0 + g.beta);
    const double eu = g.beta * el;
    const double xic = -nrep * g.dphi;

    // one azimuth xi with quadrature weight wk: the exact radial integrals
    double r0 = 0, rr = 0, rph = 0, pp = 0;
    auto point = [&](double xi, double wk) {
        double s, c;
        sincos(xi, &s, &c);
        const double sh = sin(0.5 * xi);
        double Ir = 0, Ir2 = 0, Iph = 0;
        auto f = [&](double eta, double w) {
            const double F = Fpol(eta, sh);
            const double iF3 = 1.0 / (F * F * F);
            const double fr = eta * (1.0 - eta * c) * iF3;
            Ir += w * fr;
            Ir2 += w * eta * fr;
            Iph += w * eta * eta * s * iF3;
        };
        graded_gl16(el, eu, c, fabs(s), f);
        const double wl = wk * (xi - xic);
        r0 += wk * Ir;
        rr += wk * (Ir2 - rho * Ir);
        rph += wl * Ir;
        pp += wl * Iph;
    };
    if (g.exact) {
        // Converged azimuthal integrals: 16-point Gauss-Legendre panels graded
        // towards the integrand's nearest singularities, where F = 0 for some
        // eta of the cell: xi = +-2i asinh(|eta - 1| / (2 sqrt(eta))), closest
        // for the eta of [el, eu] nearest to 1.
        const double es = fmin(fmax(1.0, el), eu);
        const double dxi = 2.0 * asinh(fabs(es - 1.0) / (2.0 * sqrt(es)));
        graded_gl16(xic - 0.5 * g.dphi, xic + 0.5 * g.dphi, 0.0, dxi, point);
    } else {
        // Eq. 41-43: n_tpz trapezoids, the weight (xi - xi_c) inside
        const double dth = g.dphi / g.n_tpz;
        for (int k = 0; k <= g.n_tpz; ++k)
            point(xic - 0.5 * g.dphi + k * dth, (k == 0 || k == g.n_tpz) ? 0.5 * dth : dth);
    }
    t[0] = -r0;
    t[1] = -rr;
    t[2] = -rph;
    t[5] = pp;

    // exact K^{phi,0}, K^{phi,r}
    const double sxc = sin(xic);
    if (sxc == 0.0) {
        t[3] = 0.0;
        t[4] = 0.0;
        return;
    }
    const double xl = xic - 0.5 * g.dphi, xu = xic + 0.5 * g.dphi;
    const double shl = sin(0.5 * xl), shu = sin(0.5 * xu);
    const double num = 4.0 * sxc * sin(0.5 * g.dphi);
    double sl, cl, su, cu;
    sincos(xl, &sl, &cl);
    sincos(xu, &su, &cu);
    // grade towards the nearer of the two unit-circle singularities
    const double mid = 0.5 * (el + eu);
    const bool lower = hypot(mid - cl, sl) <= hypot(mid - cu, su);
    double a0 = 0, a1 = 0;
    auto f2 = [&](double eta, double w) {
        const double Fl = Fpol(eta, shl), Fu = Fpol(eta, shu);
        const double D = num * eta / (Fl * Fu * (Fl + Fu));
        a0 += w * eta * D;
        a1 += w * eta * (eta - rho) * D;
    };
    graded_gl16(el, eu, lower ? cl : cu, lower ? fabs(sl) : fabs(su), f2);
    t[3] = a0;
    t[4] = a1;
}

// tables: [6][L][n_phi] FP64, row (m' mod L) for the row offset
// m' = i - i' in [-(n_in - 1), n_r - 1] between destination row i and source
// row i' (the kernel of the grid offset m = m' - s0).  One thread per
// (m', n_rep), n_rep in [0, n_phi/2]; entries at -n_rep follow from the
// parity in xi.
__global__ void k_tables(TabGeo g, const double *__restrict__ selfk, double *__restrict__ tab) {
    const int nh = g.n_phi / 2 + 1;
    const int rows = g.n_in + g.n_r - 1;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)rows * nh) return;
    const int ir = (int)(idx / nh), nrep = (int)(idx % nh);
    const int mp = ir - (g.n_in - 1);
    const int m = mp - g.s0;
    double t[6];
    if (g.method == PF_METHOD_SIM)
        table_entry(g, m, nrep, selfk, t);
    else
        particle_entry(g, m, nrep, selfk, t);
    const int row = (mp % g.L + g.L) % g.L;
    const long plane = (long)g.L * g.n_phi;
    const int cp = nrep, cn = (g.n_phi - nrep) % g.n_phi;
    const double par[6] = {1, 1, -1, -1, -1, 1};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        tab[k * plane + (long)row * g.n_phi + cp] = t[k];
        if (cn != cp) tab[k * plane + (long)row * g.n_phi + cn] = par[k] * t[k];
    }
}

__global__ void k_fill(double *__restrict__ p, long n, double v) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Self cell: Cartesian cover.
// ---------------------------------------------------------------------------
struct CoverGeo {
    double rin, rout, hx, hy, tanh_;
    long kx0, nkx, ky1, nky;
    long ncell;
    int chunk;
};

__device__ __forceinline__ double ln_plus(double y, double x, double rho) {
    // ln(y + sqrt(x^2 + y^2)); rationalised for y < 0
    return y >= 0.0 ? log(y + rho) : log(x * x / (rho - y));
}

__device__ __forceinline__ void two_sum(double &s, double &c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// Contribution of one cover cell centred at (1 + X, Y) to the three sums.
__device__ void cover_cell(const CoverGeo &g, double X, double Y, double out[3]) {
    const double xc = 1.0 + X, yc = Y;
    const double r2 = xc * xc + yc * yc;
    out[0] = out[1] = out[2] = 0.0;
    if (r2 < g.rin * g.rin || r2 > g.rout * g.rout) return;
    if (fabs(yc) > xc * g.tanh_) return;
    const double rc = sqrt(r2);
    const double s2 = rc - 1.0, ax2 = xc / rc, ay2 = yc / rc;      // rbar - 1
    const double s3 = atan2(yc, xc), ax3 = -yc / r2, ay3 = xc / r2; // phibar
    const double hmax = fmax(g.hx, g.hy);
    if (hypot(X, Y) <= 6.0 * hmax) {
        // closed forms A8-A13, evaluated at the four corners
        const double xs[2] = {X - 0.5 * g.hx, X + 0.5 * g.hx};
        const double ys[2] = {Y - 0.5 * g.hy, Y + 0.5 * g.hy};
        double ly = 0, lx = 0, ylx = 0, xly = 0, rr = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const double sg = (a == b) ? 1.0 : -1.0;
                const double x = xs[a], y = ys[b];
                const double rho = sqrt(x * x + y * y);
                const double Ly = ln_plus(y, x, rho), Lx = ln_plus(x, y, rho);
                ly += sg * Ly;
                lx += sg * Lx;
                ylx += sg * y * Lx;
                xly += sg * x * Ly;
                rr += sg * rho;
            }
        const double Kx0 = -ly, Ky0 = -lx;
        const double Kxx = -X * Kx0 + ylx, Kxy = -Y * Kx0 - rr;
        const double Kyy = -Y * Ky0 + xly, Kyx = -X * Ky0 - rr;
        out[0] = Kx0;
        out[1] = s2 * Kx0 + ax2 * Kxx + ay2 * Kxy;
        out[2] = s3 * Ky0 + ay3 * Kyy + ax3 * Kyx;
        return;
    }
    // 8 x 8 Gauss-Legendre of kernel x linear cell density (Eq. 8)
    double a1 = 0, a2 = 0, a3 = 0;
    for (int p = 0; p < 8; ++p) {
        const double u = 0.5 * g.hx * (p < 4 ? -kGL8x[3 - p] : kGL8x[p - 4]);
        const double wu = p < 4 ? kGL8w[3 - p] : kGL8w[p - 4];
        const double xb = X + u;
        double t1 = 0, t2 = 0, t3 = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double v = 0.5 * g.hy * (q < 4 ? -kGL8x[3 - q] : kGL8x[q - 4]);
            const double wv = q < 4 ? kGL8w[3 - q] : kGL8w[q - 4];
            const double yb = Y + v;
            const double rho2 = xb * xb + yb * yb;
            const double ir3 = 1.0 / (rho2 * sqrt(rho2));
            t1 += wv * xb * ir3;
            t2 += wv * xb * ir3 * (s2 + ax2 * u + ay2 * v);
            t3 += wv * yb * ir3 * (s3 + ax3 * u + ay3 * v);
        }
        a1 += wu * t1;
        a2 += wu * t2;
        a3 += wu * t3;
    }
    const double jac = 0.25 * g.hx * g.hy;
    out[0] = a1 * jac;
    out[1] = a2 * jac;
    out[2] = a3 * jac;
}

// partial[b*6 + 2q + {0,1}] = compensated (sum, carry) of quantity q.
__global__ __launch_bounds__(256) void k_cover(CoverGeo g, double *__restrict__ partial) {
    __shared__ double sh[6][256];
    double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long c0 = tid * g.chunk;
    for (int j = 0; j < g.chunk; ++j) {
        const long cell = c0 + j;
        if (cell >= g.ncell) break;
        const long kx = g.kx0 + cell / g.nky;
        const long ky = -g.ky1 + cell % g.nky;
        double o[3];
        cover_cell(g, kx * g.hx, ky * g.hy, o);
#pragma unroll
        for (int q = 0; q < 3; ++q) two_sum(s[q], c[q], o[q]);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        sh[2 * q][threadIdx.x] = s[q];
        sh[2 * q + 1][threadIdx.x] = c[q];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double ss = sh[2 * q][threadIdx.x], cc = sh[2 * q + 1][threadIdx.x];
                two_sum(ss, cc, sh[2 * q][threadIdx.x + w]);
                cc += sh[2 * q + 1][threadIdx.x + w];
                sh[2 * q][threadIdx.x] = ss;
                sh[2 * q + 1][threadIdx.x] = cc;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[(long)blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// One block folds the per-block partials into the three constants.
__global__ __launch_bounds__(256) void k_cover_final(const double *__restrict__ partial,
                                                     int nblk, double *__restrict__ selfk) {
    __shared__ double sh[6][256];
    double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            two_sum(s[q], c[q], partial[(long)b * 6 + 2 * q]);
            c[q] += partial[(long)b * 6 + 2 * q + 1];
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        sh[2 * q][threadIdx.x] = s[q];
        sh[2 * q + 1][threadIdx.x] = c[q];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double ss = sh[2 * q][threadIdx.x], cc = sh[2 * q + 1][threadIdx.x];
                two_sum(ss, cc, sh[2 * q][threadIdx.x + w]);
                cc += sh[2 * q + 1][threadIdx.x + w];
                sh[2 * q][threadIdx.x] = ss;
                sh[2 * q + 1][threadIdx.x] = cc;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        selfk[0] = sh[0][0] + sh[1][0];   // K^{r,0}_{00}
        selfk[1] = sh[2][0] + sh[3][0];   // K^{r,r}_{00} (r_m = 1, Eq. 46)
        selfk[2] = sh[4][0] + sh[5][0];   // K^{phi,phi}_{00}
    }
}

// ---------------------------------------------------------------------------
// Self cell as the exact integrals.  In local polar coordinates (rho, t)
// about the cell centre x = (1, 0), xbar = x + rho (cos t, sin t), rho up to
// the fan's boundary rho_max(t) (from Eq. 30-32 with eta deta dxi = dA):
//   K^{r,0}_{00}     = int cos t ln rho_max(t) dt       (principal value)
//   K^{r,r}_{00}     = int cos t int_0^rho_max (|xbar| - 1)/rho drho dt
//   K^{phi,phi}_{00} = int sin t int_0^rho_max phi(xbar)/rho drho dt.
// The t-range is cut at the four corner directions (rho_max has kinks
// there) and at the two directions tangent to the inner circle (where the
// ray stops meeting the inner arc, rho_max jumps when the tangent point lies
// on the cell's inner arc, and has a square-root branch point otherwise),
// and each arc takes 16-point
// Gauss-Legendre panels graded geometrically towards both of its ends
// (widths halving kPvLevels times from the middle), which converges
// exponentially whatever the singularity beyond an end.  The inner
// integrals take 16-point Gauss-Legendre on [0, rho_max] (analytic
// integrands whose singularities lie at |rho| = 1, far beyond rho_max).
// One workgroup.
// ---------------------------------------------------------------------------
struct FanGeo {
    double rin, rout, a;
    double brk[8];   // sorted break points of [0, 2 pi]
    int nb;
};

__device__ double fan_rho_max(const FanGeo &f, double t) {
    double s, c;
    sincos(t, &s, &c);
    double best = -c + sqrt(c * c + f.rout * f.rout - 1.0);
    const double disc = c * c - (1.0 - f.rin * f.rin);
    if (disc >= 0.0) {
        const double q = sqrt(disc);
        if (-c - q > 0.0 && -c - q < best) best = -c - q;
        if (-c + q > 0.0 && -c + q < best) best = -c + q;
    }
    for (int sg = -1; sg <= 1; sg += 2) {
        double ss, cs;
        sincos(sg * f.a, &ss, &cs);
        const double den = s * cs - c * ss;
        if (den != 0.0) {
            const double rr = ss / den;
            if (rr > 0.0 && rr < best) best = rr;
        }
    }
    return best;
}

constexpr int kPvLevels = 30;                  // panels per half arc
constexpr int kPvPanels = 2 * kPvLevels;       // per arc

// panel j of an arc of length len starting at lo: the half [lo, lo + len/2]
// is cut at lo + len 2^-(k+1), k = 0..kPvLevels-1 (the last panel reaching
// the end), the other half mirrored
__device__ __forceinline__ void pv_panel(double lo, double len, int j, double &a, double &b) {
    const int k = j < kPvLevels ? j : kPvPanels - 1 - j;   // level from the middle
    const double outer = ldexp(len, -(k + 1));              // distance of the panel's
    const double inner = k + 1 < kPvLevels ? ldexp(len, -(k + 2)) : 0.0;   // edges to the end
    if (j < kPvLevels) {
        a = lo + inner;
        b = lo + outer;
    } else {
        a = lo + len - outer;
        b = lo + len - inner;
    }
}

__global__ __launch_bounds__(256) void k_selfpv(FanGeo f, double *__restrict__ out) {
    __shared__ double sh[3][256];
    const int total = (f.nb - 1) * kPvPanels * 16;
    double k0 = 0.0, k1 = 0.0, k2 = 0.0;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int arc = idx / (kPvPanels * 16), rem = idx % (kPvPanels * 16);
        const int pnl = rem / 16, q = rem % 16;
        double pa, pb;
        pv_panel(f.brk[arc], f.brk[arc + 1] - f.brk[arc], pnl, pa, pb);
        const double width = pb - pa;
        const double mid = 0.5 * (pa + pb);
        const double xq = (q < 8 ? -1.0 : 1.0) * kGL16x[q & 7];
        const double t = mid + 0.5 * width * xq, wt = 0.5 * width * kGL16w[q & 7];
        double s, c;
        sincos(t, &s, &c);
        const double rm = fan_rho_max(f, t);
        double a = 0.0, b = 0.0;
        for (int j = 0; j < 16; ++j) {
            const double rho = 0.5 * rm * (1.0 + (j < 8 ? -1.0 : 1.0) * kGL16x[j & 7]);
            const double X = 1.0 + rho * c, Y = rho * s;
            const double R = sqrt(X * X + Y * Y);
            a += kGL16w[j & 7] * (2.0 * c + rho) / (R + 1.0);   // (|xbar| - 1) / rho
            b += kGL16w[j & 7] * atan2(Y, X) / rho;
        }
        k0 += wt * c * log(rm);
        k1 += wt * c * 0.5 * rm * a;
        k2 += wt * s * 0.5 * rm * b;
    }
    sh[0][threadIdx.x] = k0;
    sh[1][threadIdx.x] = k1;
    sh[2][threadIdx.x] = k2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] = sh[k][0];
}

// ---------------------------------------------------------------------------
// Column transforms of the row-transformed tables and the fold into the four
// spectra.  rowspec: [6][L][M] complex FP64 in the packed half spectrum
// (column 0 = (bin 0, bin M)).  spec: [2][M][ldspec] pairs (E', Q).
// One block per azimuthal bin kb in [0, M] (bins 0 and M read the real and
// imaginary parts of packed column 0), L/E threads.  With s = 1/(L n_phi),
// sk = sin(2 pi kb / n_phi) / dphi (the azimuthal central difference) and
// D(k) = 2i ca sin(2 pi k / L) (the circular radial central difference);
// for slope order 4 the five-point differences,
// sk = (8 sin(2 pi kb / n_phi) - sin(4 pi kb / n_phi)) / (6 dphi) and
// D(k) = 2i c4 (8 sin(2 pi k / L) - sin(4 pi k / L)):
//   Q_r  = s FFT(beta^m T_rr)         E_r = s (FFT(T_r0) + i sk FFT(T_rphi))
//   Q_p  = s FFT(beta^m T_phir)       E_p = s (FFT(T_phi0) + i sk FFT(T_phiphi))
//   E'   = E + D Q
// Bins 1..M-1 store the pairs (E'_r, Q_r) and (E'_p, Q_p) in their column;
// column 0 holds the radial pair of bin 0 first and that of bin M second
// (the azimuthal spectra vanish at both: the kernels K^{phi,*} are odd in
// phi).
// ---------------------------------------------------------------------------
template <int L, int E>
__global__ __launch_bounds__(512) void k_fold(const cx<double> *__restrict__ rowspec, int M,
                                              int n_r, int s0, int n_phi, double lnb,
                                              double dphi, double ca,
                                              cx2<double> *__restrict__ spec, int ldspec,
                                              const cx<double> *__restrict__ twL, int so,
                                              double c4) {
    constexpr int TH = L / E;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double> *buf = reinterpret_cast<cx<double> *>(smem_raw);
    const int kb = blockIdx.x, t = threadIdx.x;
    const int src = kb == M ? 0 : kb;
    const int part = kb == 0 ? 1 : (kb == M ? 2 : 0);   // 1: real, 2: imaginary part of column 0
    Lds<double> lds{buf, 0, 1};
    Twiddles<L, E, double> tw;
    tw.load(t, twL, 1);
    const double sc = 1.0 / ((double)L * (double)n_phi);
    const double sk = so == 4 ? (8.0 * sinpi(2.0 * kb / n_phi) - sinpi(4.0 * kb / n_phi)) / (6.0 * dphi)
                              : sinpi(2.0 * kb / n_phi) / dphi;

    auto load = [&](int tab, bool bscale, cx<double>(&v)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = t + e * TH;
            cx<double> x = rowspec[((size_t)tab * L + row) * M + src];
            if (part == 1) x = cx<double>{x.x, 0.0};
            if (part == 2) x = cx<double>{x.y, 0.0};
            if (bscale) {   // r_i / r_i' = beta^m, m = m' - s0 the grid offset
                const int mp = row < n_r ? row : row - L;
                x = scale(x, exp((mp - s0) * lnb));
            }
            v[e] = x;
        }
        fft_fwd<L, E, double>(v, t, lds, tw);
    };
    auto store = [&](int pair, const cx<double>(&ev)[E], const cx<double>(&qv)[E]) {
        cx2<double> *dst = spec + ((size_t)pair * M + src) * ldspec;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ku = t + e * TH;
            if (ku <= L / 2) dst[ku] = cx2<double>{ev[e], qv[e]};
        }
    };
    // (E', Q) of one channel from the tables (t0, tr, tphi)
    auto channel = [&](int t0, int tr, int tphi, int pair) {
        cx<double> q[E], a[E], b[E];
        load(tr, true, q);
        load(t0, false, a);
        load(tphi, false, b);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ku = t + e * TH;
            const double d = so == 4 ? 2.0 * c4 * (8.0 * sinpi(2.0 * ku / L) - sinpi(4.0 * ku / L))
                                     : 2.0 * ca * sinpi(2.0 * ku / L);
            const cx<double> qe = scale(q[e], sc);
            const cx<double> ee = {(a[e].x - sk * b[e].y) * sc, (a[e].y + sk * b[e].x) * sc};
            a[e] = cx<double>{ee.x - d * qe.y, ee.y + d * qe.x};   // E + i d Q
            q[e] = qe;
        }
        store(pair, a, q);
    };
    if (part == 2)
        channel(0, 1, 2, 1);       // bin M's radial pair into column 0's second pair
    else
        channel(0, 1, 2, 0);
    if (part == 0) channel(3, 4, 5, 1);
}

__global__ void k_to_f32(const cx<double> *__restrict__ in, cx<float> *__restrict__ out, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        out[i] = cx<float>{(float)in[i].x, (float)in[i].y};
}

namespace {

template <int L, int E>
int fold_launch(const cx<double> *rowspec, const Plan &p, cx2<double> *spec,
                const cx<double> *twL, hipStream_t st) {
    if constexpr (E <= L) {
        const size_t lds = (size_t)padded_len(L) * sizeof(cx<double>);
        if (lds > 64 * 1024)
            PF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_fold<L, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((k_fold<L, E>), dim3(p.M + 1), dim3(L / E), lds, st, rowspec, p.M,
                           p.n_r, p.s0, p.n_phi, std::log(p.beta), p.dphi, p.ca, spec,
                           p.ldspec, twL, p.so, p.c4);
        PF_HIP(hipGetLastError());
        return PF_OK;
    }
    set_error("fold: bad size");
    return PF_EUNSUPPORTED;
}

int fold_dispatch(const cx<double> *rowspec, const Plan &p, cx2<double> *spec,
                  const cx<double> *twL, hipStream_t st) {
    switch (p.L) {
        case 8: return fold_launch<8, 8>(rowspec, p, spec, twL, st);
        case 16: return fold_launch<16, 8>(rowspec, p, spec, twL, st);
        case 32: return fold_launch<32, 8>(rowspec, p, spec, twL, st);
        case 64: return fold_launch<64, 8>(rowspec, p, spec, twL, st);
        case 128: return fold_launch<128, 8>(rowspec, p, spec, twL, st);
        case 256: return fold_launch<256, 8>(rowspec, p, spec, twL, st);
        case 512: return fold_launch<512, 8>(rowspec, p, spec, twL, st);
        case 1024: return fold_launch<1024, 8>(rowspec, p, spec, twL, st);
        case 2048: return fold_launch<2048, 8>(rowspec, p, spec, twL, st);
        case 4096: return fold_launch<4096, 16>(rowspec, p, spec, twL, st);
        case 8192: return fold_launch<8192, 16>(rowspec, p, spec, twL, st);
    }
    set_error("fold: unsupported L=%d", p.L);
    return PF_EUNSUPPORTED;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

int build_tables_and_spectra(Plan &p, hipStream_t st) {
    const bool f64 = p.opts.dtype == PF_F64;
    const long plane = (long)p.L * p.n_phi;
    DevBuf tab, rowspec, spec64, selfk, partial, twN64, twL64;

    // --- self cell by the Cartesian cover ---------------------------------
    CoverGeo cg{};
    {
        const double beta = p.beta, dphi = p.dphi;
        const double dr = 2.0 * (beta - 1.0) / (1.0 + beta);
        cg.rin = 1.0 - 0.5 * dr;
        cg.rout = 1.0 + 0.5 * dr;
        const double sq = std::sin(0.25 * dphi);
        const double Dx = cg.rin * 2.0 * sq * sq;        // (r_m - dr/2)(1 - cos(dphi/2))
        const double Dy = dr * std::sin(0.5 * dphi);     // dr sin(dphi/2)
        cg.hx = Dx / p.opts.cover_per;
        cg.hy = Dy / p.opts.cover_per;
        const double ch = std::cos(0.5 * dphi), shf = std::sin(0.5 * dphi);
        cg.tanh_ = shf / ch;
        cg.kx0 = (long)std::ceil((cg.rin * ch - 1.0) / cg.hx);
        const long kx1 = (long)std::floor((cg.rout - 1.0) / cg.hx);
        cg.ky1 = (long)std::floor(cg.rout * shf / cg.hy);
        cg.nkx = kx1 - cg.kx0 + 1;
        cg.nky = 2 * cg.ky1 + 1;
        cg.ncell = cg.nkx * cg.nky;
        cg.chunk = 16;
    }
    PF_HIP(hipMalloc(&selfk.p, 3 * sizeof(double)));
    if (p.opts.self_mode == PF_SELF_EXACT) {
        FanGeo fg{};
        fg.rin = 2.0 / (1.0 + p.beta);
        fg.rout = 2.0 * p.beta / (1.0 + p.beta);
        fg.a = 0.5 * p.dphi;
        std::vector<double> b = {0.0, 2.0 * M_PI};
        for (double R : {fg.rin, fg.rout})
            for (double sa : {fg.a, -fg.a}) {   // corners
                double t = std::atan2(R * std::sin(sa), R * std::cos(sa) - 1.0);
                if (t < 0.0) t += 2.0 * M_PI;
                b.push_back(t);
            }
        for (double sg : {1.0, -1.0}) {   // tangents to the inner circle
            const double ty = sg * fg.rin * std::sqrt(1.0 - fg.rin * fg.rin);
            double t = std::atan2(ty, fg.rin * fg.rin - 1.0);
            if (t < 0.0) t += 2.0 * M_PI;
            b.push_back(t);
        }
        std::sort(b.begin(), b.end());
        fg.nb = (int)b.size();
        for (int k = 0; k < fg.nb; ++k) fg.brk[k] = b[k];
        hipLaunchKernelGGL(k_selfpv, dim3(1), dim3(256), 0, st, fg, (double *)selfk.p);
        PF_HIP(hipGetLastError());
    } else {
        const long nthreads = (cg.ncell + cg.chunk - 1) / cg.chunk;
        const int nblk = (int)((nthreads + 255) / 256);
        PF_HIP(hipMalloc(&partial.p, (size_t)nblk * 6 * sizeof(double)));
        hipLaunchKernelGGL(k_cover, dim3(nblk), dim3(256), 0, st, cg, (double *)partial.p);
        PF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_cover_final, dim3(1), dim3(256), 0, st, (const double *)partial.p,
                           nblk, (double *)selfk.p);
        PF_HIP(hipGetLastError());
    }

    // --- kernel tables -------------------------------------------------------
    PF_HIP(hipMalloc(&tab.p, 6 * plane * sizeof(double)));
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, st, (double *)tab.p, 6 * plane, 0.0);
    PF_HIP(hipGetLastError());
    TabGeo tg{p.beta, p.dphi, std::log(p.beta), p.n_r, p.n_phi, p.L, p.opts.n_tpz,
              p.opts.table_mode == PF_TABLE_EXACT ? 1 : 0, p.opts.method, p.n_in, p.s0};
    {
        const long n = (long)(p.n_in + p.n_r - 1) * (p.n_phi / 2 + 1);
        hipLaunchKernelGGL(k_tables, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, tg,
                           (const double *)selfk.p, (double *)tab.p);
        PF_HIP(hipGetLastError());
    }

    // --- spectra ---------------------------------------------------------------
    int rc = upload_twiddles(p.n_phi, true, &twN64.p);
    if (rc) return rc;
    rc = upload_twiddles(p.L, true, &twL64.p);
    if (rc) return rc;
    PF_HIP(hipMalloc(&rowspec.p, (size_t)6 * p.L * p.M * sizeof(cx<double>)));
    {
        Shape s = default_schedule(p.n_phi, p.L, true).rows;
        rc = launch_rows_r2c<double>(p, (const double *)tab.p, nullptr, 6 * p.L,
                                     (cx<double> *)rowspec.p, (const cx<double> *)twN64.p, s,
                                     st);
        if (rc) return rc;
    }
    const size_t nspec = (size_t)4 * p.M * p.ldspec;
    PF_HIP(hipMalloc(&spec64.p, nspec * sizeof(cx<double>) + kSpecTailPad));
    rc = fold_dispatch((const cx<double> *)rowspec.p, p, (cx2<double> *)spec64.p,
                       (const cx<double> *)twL64.p, st);
    if (rc) return rc;

    void *spec_final = nullptr;
    if (f64) {
        spec_final = spec64.p;
        spec64.p = nullptr;
    } else {
        PF_HIP(hipMalloc(&spec_final, nspec * sizeof(cx<float>) + kSpecTailPad));
        hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, st, (const cx<double> *)spec64.p,
                           (cx<float> *)spec_final, (long)nspec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipFree(spec_final);
            set_error("k_to_f32: %s", hipGetErrorString(e));
            return PF_EHIP;
        }
    }
    double hk[3];
    hipError_t e = hipMemcpyAsync(hk, selfk.p, sizeof(hk), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(spec_final);
        set_error("table build: %s", hipGetErrorString(e));
        return PF_EHIP;
    }
    if (p.spec) (void)hipFree(p.spec);
    p.spec = spec_final;
    for (int q = 0; q < 3; ++q) p.selfk[q] = hk[q];
    if (p.tables) {
        (void)hipFree(p.tables);
        p.tables = nullptr;
    }
    if (p.opts.keep_tables) {
        p.tables = (double *)tab.p;
        tab.p = nullptr;
    }
    return PF_OK;
}

// ---------------------------------------------------------------------------
// Origin wedges: the cells [0, r_w] x [phi_j' +- dphi/2], r_w = r_min beta^s0,
// below the source rows (Sec. 3.2.1; the paper uses barred kernels for them
// without defining them).  Reading: the integrands of Eq. 30-32 and A22-A24
// over the wedge, with the wedge's radial centre at r_w / 2 (the arithmetic
// centre, as for every other cell); in units of r_i (eta = rbar / r_i,
// eta_w = r_w / r_i, eta_c = eta_w / 2, xi_c = -n dphi)
//   T_r0 = -int eta (1 - eta cos xi) / F^3,      T_phi0 = int eta^2 sin xi / F^3,
//   T_rr = -int eta (1 - eta cos xi) (eta - eta_c) / F^3, T_phir likewise,
//   T_rphi = -int eta (1 - eta cos xi) (xi - xi_c) / F^3, T_phiphi likewise,
// over eta in [0, eta_w], xi in [xi_c +- dphi/2]; the particle methods take
// the wedge as the point mass sigma r_w^2 dphi / 2 at (r_w / 2, phi_j').
// Radial integrals by 16-point Gauss-Legendre graded towards the complex
// zeros of F for each azimuth, the azimuthal integral graded towards
// xi = +-i 2 asinh((1 - eta_w) / (2 sqrt(eta_w))), where F vanishes at the
// wedge's outer edge.  The wedges act on row i through a periodic
// convolution in phi only; F^r += sigma T_r0 + r_i delta^r T_rr +
// delta^phi T_rphi (and likewise F^phi), with the wedge's azimuthal slope by
// periodic central differences and its radial slope by the one-sided
// difference towards the first source row.
// ---------------------------------------------------------------------------
struct WedgeGeo {
    double beta, dphi, r_min;
    int n_r, n_phi, s0, method;
};

// tab: [6][n_r][n_phi], column n = (j - j') mod n_phi
__global__ void k_wedge_tables(WedgeGeo g, double *__restrict__ tab) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)g.n_r * g.n_phi) return;
    const int i = (int)(idx / g.n_phi), n = (int)(idx % g.n_phi);
    const int nrep = n <= g.n_phi / 2 ? n : n - g.n_phi;
    const double xic = -nrep * g.dphi;
    const double ri = g.r_min * pow(g.beta, (double)i) * 0.5 * (1.0 + g.beta);
    const double ew = g.r_min * pow(g.beta, (double)g.s0) / ri;
    const double ec = 0.5 * ew;
    double t[6] = {0, 0, 0, 0, 0, 0};
    if (g.method == PF_METHOD_SIM) {
        double a[6] = {0, 0, 0, 0, 0, 0};
        auto point = [&](double xi, double wk) {
            double sx, cxi;
            sincos(xi, &sx, &cxi);
            const double sh = sin(0.5 * xi);
            double ir = 0, ir2 = 0, ip = 0, ip2 = 0;
            auto f = [&](double eta, double w) {
                const double F = Fpol(eta, sh);
                const double iF3 = 1.0 / (F * F * F);
                const double fr = eta * (1.0 - eta * cxi) * iF3;
                const double fp = eta * eta * sx * iF3;
                ir += w * fr;
                ir2 += w * fr * (eta - ec);
                ip += w * fp;
                ip2 += w * fp * (eta - ec);
            };
            graded_gl16(0.0, ew, cxi, fabs(sx), f);
            const double wl = wk * (xi - xic);
            a[0] += wk * ir;
            a[1] += wk * ir2;
            a[2] += wl * ir;
            a[3] += wk * ip;
            a[4] += wk * ip2;
            a[5] += wl * ip;
        };
        const double dxi = 2.0 * asinh((1.0 - ew) / (2.0 * sqrt(ew)));
        graded_gl16(xic - 0.5 * g.dphi, xic + 0.5 * g.dphi, 0.0, dxi, point);
        t[0] = -a[0];
        t[1] = -a[1];
        t[2] = -a[2];
        t[3] = a[3];
        t[4] = a[4];
        t[5] = a[5];
    } else {
        const double A = 0.5 * ew * ew * g.dphi;
        const double F = Fpol(ec, sin(0.5 * xic));
        const double iF3 = 1.0 / (F * F * F);
        double sx, cxi;
        sincos(xic, &sx, &cxi);
        t[0] = A * (ec * cxi - 1.0) * iF3;
        t[3] = A * ec * sx * iF3;
    }
    const size_t plane = (size_t)g.n_r * g.n_phi;
#pragma unroll
    for (int k = 0; k < 6; ++k) tab[k * plane + (size_t)i * g.n_phi + n] = t[k];
}

// Wedge spectra per destination row: wspec[c][i][k], pairs (E, Q) with
//   E = s (T_0 + i sk T_phi),  Q = s r_i T_r,   s = 1 / n_phi,
// sk = sin(2 pi k / n_phi) / dphi; c = 0 the radial force, c = 1 the
// azimuthal one; column 0 holds the radial pair of bin 0 (c = 0) and of
// bin n_phi/2 (c = 1), the azimuthal spectra vanishing at both.
__global__ void k_wedge_fold(const cx<double> *__restrict__ rowspec, WedgeGeo g, int H,
                             cx2<double> *__restrict__ wspec) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)g.n_r * (H + 1)) return;
    const int i = (int)(idx / (H + 1)), kb = (int)(idx % (H + 1));
    const int src = kb == H ? 0 : kb;
    const int part = kb == 0 ? 1 : (kb == H ? 2 : 0);
    auto get = [&](int tab) {
        cx<double> x = rowspec[((size_t)tab * g.n_r + i) * H + src];
        if (part == 1) x = cx<double>{x.x, 0.0};
        if (part == 2) x = cx<double>{x.y, 0.0};
        return x;
    };
    const double sw = 1.0 / g.n_phi;
    const double sk = sinpi(2.0 * kb / g.n_phi) / g.dphi;
    const double ri = g.r_min * pow(g.beta, (double)i) * 0.5 * (1.0 + g.beta);
    auto pair = [&](int t0, int tr, int tp) {
        const cx<double> a = get(t0), b = get(tp), q = get(tr);
        return cx2<double>{{(a.x - sk * b.y) * sw, (a.y + sk * b.x) * sw}, scale(q, sw * ri)};
    };
    if (part == 0) {
        wspec[(size_t)i * H + kb] = pair(0, 1, 2);
        wspec[((size_t)g.n_r + i) * H + kb] = pair(3, 4, 5);
    } else {
        wspec[((size_t)(part == 1 ? 0 : g.n_r) + i) * H] = pair(0, 1, 2);
    }
}

// Z[i][k] += wedge terms.  w[k] = sigma_w^ (the wedge row's spectrum); the
// wedges' radial slope (sigma_src[0] - sigma_w) / (r_0 - r_w / 2) is linear,
// so its spectrum is (S[0][k] - w[k]) inv_dr with S[0] the first source
// row's spectrum from pass A (bins 0 and n_phi/2 packed alike).
template <typename T>
__global__ void k_wedge_add(cx2<T> *__restrict__ Z, const cx2<T> *__restrict__ wspec,
                            const cx<T> *__restrict__ w, const cx<T> *__restrict__ S0,
                            T inv_dr, int n_r, int H, const unsigned *__restrict__ g) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n_r * H) return;
    const int k = (int)(idx % H);
    const cx2<T> a = wspec[idx], b = wspec[(size_t)n_r * H + idx];
    cx<T> ws = w[k], s0 = S0[k];
    if (g) {
        // FP32 calls: Z holds the column pass's output scaled by 2^-e (e in
        // the scale words, after the 64 notes); the wedge terms join it at
        // the same scale, applied before the slope's 1 / (r_0 - r_w / 2) so
        // that no unscaled product leaves the range
        const int ex = (int)g[kScaleE];
        const T s = (T)__uint_as_float((unsigned)(127 - ex) << 23);
        ws = scale(ws, s);
        s0 = scale(s0, s);
    }
    const cx2<T> x = {ws, scale(s0 - ws, inv_dr)};
    cx2<T> z = Z[idx];
    if (k == 0) {   // bins 0 and n_phi/2: real parts, radial force only
        z.a.x += a.a.x * x.a.x + a.b.x * x.b.x;
        z.a.y += b.a.x * x.a.y + b.b.x * x.b.y;
    } else {
        z.a = z.a + cmul(a.a, x.a) + cmul(a.b, x.b);
        z.b = z.b + cmul(b.a, x.a) + cmul(b.b, x.b);
    }
    Z[idx] = z;
}

// Transpose of the wedge terms.  The forward adds A[i][k] w[k] (radial) and
// B[i][k] w[k] (azimuthal) to row i's spectra, w = (sigma_w^, delta^r^);
// its transpose takes the cotangents' row spectra V[i][k] = (V_r, V_p) to
//   wbar[k] = sum over destination rows i of conj(A) V_r + conj(B) V_p
// (pair by pair: the sigma_w part and the delta^r part), bins 0 and
// n_phi/2 real and packed as in the forward.  Stage 1: workgroup (x, y)
// sums the rows of chunk y for bins [64 x, 64 x + 64), four row lanes per
// bin, reduced through LDS in a fixed order; stage 2 sums the chunks in
// order, so the result does not depend on timing, and splits wbar into
// the wedge row's spectrum and the first source row's share.  FP32: V is
// the pass-A output (unscaled); it is taken times 2^-e (e from the
// transpose's scale words, written by its column pass), so wbar carries the
// same scale as the column pass's output D, and the row transforms that
// follow (pass C, the wedge row's) restore it.
constexpr int kWedgeLanes = 4;
template <typename T>
__global__ __launch_bounds__(64 * kWedgeLanes) void k_wedge_adj_part(
    const cx2<T> *__restrict__ V, const cx2<T> *__restrict__ wspec, int n_r, int H, int rows,
    cx2<T> *__restrict__ part, const unsigned *__restrict__ g) {
    const int k = blockIdx.x * 64 + (threadIdx.x & 63);
    const int lane = threadIdx.x >> 6;
    const int i0 = blockIdx.y * rows, i1 = min(n_r, i0 + rows);
    T s = T(1);
    if (g) {
        const int ex = (int)g[kScaleE];
        s = (T)__uint_as_float((unsigned)(127 - ex) << 23);
    }
    cx2<T> acc = {{T(0), T(0)}, {T(0), T(0)}};
    if (k < H) {
        for (int i = i0 + lane; i < i1; i += kWedgeLanes) {
            const size_t idx = (size_t)i * H + k;
            const cx2<T> a = wspec[idx], b = wspec[(size_t)n_r * H + idx];
            cx2<T> v = V[idx];
            v = cx2<T>{scale(v.a, s), scale(v.b, s)};
            if (k == 0) {   // bins 0 and n_phi/2: real parts, radial force only
                acc.a.x = fmadd(a.a.x, v.a.x, acc.a.x);
                acc.a.y = fmadd(b.a.x, v.a.y, acc.a.y);
                acc.b.x = fmadd(a.b.x, v.a.x, acc.b.x);
                acc.b.y = fmadd(b.b.x, v.a.y, acc.b.y);
            } else {
                acc.a = cmacc(cmacc(acc.a, v.a, a.a), v.b, b.a);
                acc.b = cmacc(cmacc(acc.b, v.a, a.b), v.b, b.b);
            }
        }
    }
    __shared__ cx2<T> red[kWedgeLanes][64];
    red[lane][threadIdx.x & 63] = acc;
    __syncthreads();
    if (lane == 0 && k < H) {
#pragma unroll
        for (int l = 1; l < kWedgeLanes; ++l) {
            const cx2<T> o = red[l][threadIdx.x];
            acc.a = acc.a + o.a;
            acc.b = acc.b + o.b;
        }
        part[(size_t)blockIdx.y * H + k] = acc;
    }
}

// Stage 2: wbar = (wbar_s, wbar_d) summed over the chunks: sixteen lanes per
// bin (sixteen bins per workgroup), lane l taking chunks l, l + 16, ... in
// order, then the lanes in order (a fixed order); the wedge row's spectrum
// gets wbar_s - inv_dr wbar_d (sigma_w enters its own density and,
// negatively, its radial slope) and the first source row's spectrum D[0]
// (the column pass's output, before pass C) its share of that slope,
// + inv_dr wbar_d.
constexpr int kSumLanes = 16;
template <typename T>
__global__ __launch_bounds__(16 * kSumLanes) void k_wedge_adj_sum(
    const cx2<T> *__restrict__ part, int chunks, int H, T inv_dr, cx<T> *__restrict__ wg,
    cx<T> *__restrict__ D0) {
    const int k = blockIdx.x * 16 + (threadIdx.x & 15);
    const int lane = threadIdx.x >> 4;
    cx2<T> acc = {{T(0), T(0)}, {T(0), T(0)}};
    if (k < H)
        for (int c = lane; c < chunks; c += kSumLanes) {
            const cx2<T> o = part[(size_t)c * H + k];
            acc.a = acc.a + o.a;
            acc.b = acc.b + o.b;
        }
    __shared__ cx2<T> red[kSumLanes][16];
    red[lane][threadIdx.x & 15] = acc;
    __syncthreads();
    if (lane == 0 && k < H) {
#pragma unroll
        for (int l = 1; l < kSumLanes; ++l) {
            const cx2<T> o = red[l][threadIdx.x];
            acc.a = acc.a + o.a;
            acc.b = acc.b + o.b;
        }
        const cx<T> d = scale(acc.b, inv_dr);
        wg[k] = acc.a - d;
        D0[k] = D0[k] + d;
    }
}

// Row chunks of the wedge transpose's first stage: enough workgroups to
// spread the row sums over the chip, at least four rows per lane
static void wedge_adj_chunks(int n_r, int H, int *rows, int *chunks) {
    const int bx = (H + 63) / 64;
    int c = std::max(1, std::min((1024 + bx - 1) / bx, (n_r + 4 * kWedgeLanes - 1) / (4 * kWedgeLanes)));
    *rows = (n_r + c - 1) / c;
    *chunks = (n_r + *rows - 1) / *rows;
}

int build_wedge_spectra(Plan &p, hipStream_t st) {
    const bool f64 = p.opts.dtype == PF_F64;
    DevBuf tab, rowspec, w64, twN64;
    const size_t plane = (size_t)p.n_r * p.n_phi;
    WedgeGeo g{p.beta, p.dphi, p.r_min, p.n_r, p.n_phi, p.s0,
               p.opts.method == PF_METHOD_SIM ? PF_METHOD_SIM : PF_METHOD_PARTICLE};
    PF_HIP(hipMalloc(&tab.p, 6 * plane * sizeof(double)));
    hipLaunchKernelGGL(k_wedge_tables, dim3((unsigned)((plane + 127) / 128)), dim3(128), 0, st, g,
                       (double *)tab.p);
    PF_HIP(hipGetLastError());
    int rc = upload_twiddles(p.n_phi, true, &twN64.p);
    if (rc) return rc;
    PF_HIP(hipMalloc(&rowspec.p, 6 * (size_t)p.n_r * p.H * sizeof(cx<double>)));
    rc = launch_rows_r2c<double>(p, (const double *)tab.p, nullptr, 6 * p.n_r,
                                 (cx<double> *)rowspec.p, (const cx<double> *)twN64.p,
                                 default_schedule(p.n_phi, p.L, true).rows, st);
    if (rc) return rc;
    const size_t nw = (size_t)2 * p.n_r * p.H;   // pairs
    PF_HIP(hipMalloc(&w64.p, nw * sizeof(cx2<double>)));
    {
        const long n = (long)p.n_r * (p.H + 1);
        hipLaunchKernelGGL(k_wedge_fold, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st,
                           (const cx<double> *)rowspec.p, g, p.H, (cx2<double> *)w64.p);
        PF_HIP(hipGetLastError());
    }
    if (f64) {
        p.wspec = w64.p;
        w64.p = nullptr;
    } else {
        PF_HIP(hipMalloc(&p.wspec, nw * sizeof(cx2<float>)));
        hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, st, (const cx<double> *)w64.p,
                           (cx<float> *)p.wspec, (long)(2 * nw));
        PF_HIP(hipGetLastError());
    }
    // workspace: the wedge row's spectrum (H complex), then (transpose) the
    // stage-1 partial sums (chunks x H pairs)
    int rows, chunks;
    wedge_adj_chunks(p.n_r, p.H, &rows, &chunks);
    const size_t cb = f64 ? 16 : 8;
    PF_HIP(hipMalloc(&p.wws, (size_t)p.H * cb + (size_t)chunks * p.H * 2 * cb));
    PF_HIP(hipStreamSynchronize(st));
    return PF_OK;
}

template <typename T>
int launch_wedge_terms(const Plan &p, const cx<T> *S, const cx<T> *wrow, cx<T> *Z,
                       hipStream_t st, const unsigned *g) {
    const double rc0 = p.r_min * std::pow(p.beta, p.s0) * 0.5 * (1.0 + p.beta);
    const double rh = 0.5 * p.r_min * std::pow(p.beta, p.s0);
    const long n = (long)p.n_r * p.H;
    hipLaunchKernelGGL(k_wedge_add<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<cx2<T> *>(Z), (const cx2<T> *)p.wspec, wrow, S,
                       T(1.0 / (rc0 - rh)), p.n_r, p.H, sizeof(T) == 4 ? g : nullptr);
    PF_HIP(hipGetLastError());
    return PF_OK;
}

template <typename T>
int launch_wedge_adjoint_sums(const Plan &p, const cx<T> *V, cx<T> *D, hipStream_t st,
                              unsigned *g) {
    int rows, chunks;
    wedge_adj_chunks(p.n_r, p.H, &rows, &chunks);
    cx<T> *wg = (cx<T> *)p.wws;
    cx2<T> *part = reinterpret_cast<cx2<T> *>(wg + p.H);
    const double rc0 = p.r_min * std::pow(p.beta, p.s0) * 0.5 * (1.0 + p.beta);
    const double rh = 0.5 * p.r_min * std::pow(p.beta, p.s0);
    const unsigned *gs = sizeof(T) == 4 ? g : nullptr;
    hipLaunchKernelGGL(k_wedge_adj_part<T>, dim3((unsigned)((p.H + 63) / 64), (unsigned)chunks),
                       dim3(64 * kWedgeLanes), 0, st, reinterpret_cast<const cx2<T> *>(V),
                       (const cx2<T> *)p.wspec, p.n_r, p.H, rows, part, gs);
    PF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_wedge_adj_sum<T>, dim3((unsigned)((p.H + 15) / 16)),
                       dim3(16 * kSumLanes), 0, st, (const cx2<T> *)part, chunks, p.H,
                       T(1.0 / (rc0 - rh)), wg, D);
    PF_HIP(hipGetLastError());
    return PF_OK;
}

template int launch_wedge_adjoint_sums<float>(const Plan &, const cx<float> *, cx<float> *,
                                              hipStream_t, unsigned *);
template int launch_wedge_adjoint_sums<double>(const Plan &, const cx<double> *, cx<double> *,
                                               hipStream_t, unsigned *);

template int launch_wedge_terms<float>(const Plan &, const cx<float> *, const cx<float> *,
                                       cx<float> *, hipStream_t, const unsigned *);
template int launch_wedge_terms<double>(const Plan &, const cx<double> *, const cx<double> *,
                                        cx<double> *, hipStream_t, const unsigned *);

}  // namespace pf
