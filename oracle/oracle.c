/*
 * FP64 CPU oracle for the finite-difference lattice Boltzmann (FDLB) step of the
 * simplified Enskog equation with a Shakhov collision term (Busuioc, arXiv 2211.16933).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP path
 * is checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant with the
 * GPU library: every quantity below is recomputed here from the paper's definitions.
 *
 * Units: m = k_B = 1 and T_ref = 1 (Sec. II.A, last paragraph).  rho == n.
 *
 * Storage convention used by every entry point: a distribution psi in {phi, theta} is a
 * row-major array of (nx + 6) rows by q columns.  Row r holds cell i = r - 3, so rows
 * 0..2 and nx+3..nx+5 are the three ghost cells per side needed by the +-3 stencils.
 * Values are quadrature-weighted: n = sum_k phi_k (Sec. II.D, discrete moments).
 *
 * Readings of points where the paper is silent or garbled are marked "Reading:".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_NG 3 /* ghost cells per side */

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_EROOTS = 3 };
enum { OR_PR_CONST = 0, OR_PR_ENSKOG = 1 };
enum { OR_BC_PERIODIC = 0, OR_BC_EQUILIBRIUM = 1 };
enum { OR_CHI_SET = 0, OR_CHI_RETFM = 1 };

typedef struct {
    int nx;        /* interior cells */
    int q;         /* quadrature nodes Q */
    int nh;        /* Hermite order N of the equilibrium expansion, 0 <= N <= Q-1 */
    double dx, dt; /* cell width and time step */
    double b;      /* covolume b = 2 pi sigma^3 / 3m; eta = b n / 4 */
    double mu_ref; /* dilute hard-sphere viscosity at T_0 = 1 */
    int pr_mode;   /* OR_PR_CONST: Pr = pr; OR_PR_ENSKOG: dense-gas Pr(b n chi) */
    double pr;
    int bc;        /* OR_BC_PERIODIC or OR_BC_EQUILIBRIUM (ghost rows held fixed) */
    int chi_mode;  /* OR_CHI_SET: chi_SET(n); OR_CHI_RETFM: chi_SET of the ball average */
    double sigma;  /* molecular diameter (used by OR_CHI_RETFM) */
} or_params;

/* ------------------------------------------------------------------------------------
 * Hermite polynomials and the full-range Gauss-Hermite quadrature (Sec. II.D).
 * ---------------------------------------------------------------------------------- */

/* Probabilists' Hermite polynomial He_l(x), orthogonal under exp(-x^2/2)/sqrt(2 pi),
 * from its three-term recurrence He_{l+1} = x He_l - l He_{l-1}, He_0 = 1, He_1 = x. */
double or_hermite(int l, double x)
{
    double hm = 1.0, h = x;
    if (l == 0) return 1.0;
    for (int j = 1; j < l; ++j) {
        double hp = x * h - j * hm;
        hm = h;
        h = hp;
    }
    return h;
}

/* He_l(x) / sqrt(l!), the same recurrence divided through by sqrt(l!), which keeps the
 * values finite for the large l and |x| reached when Q is large. */
static double hermite_normalised(int l, double x)
{
    double hm = 1.0, h = x;
    if (l == 0) return 1.0;
    for (int j = 1; j < l; ++j) {
        double hp = (x * h - sqrt((double)j) * hm) / sqrt((double)(j + 1));
        hm = h;
        h = hp;
    }
    return h;
}

/* Nodes p_k (ascending) are the Q roots of He_Q; the weights are
 *   w_k = Q! / [He_{Q+1}(p_k)]^2          (Sec. II.D, weight formula),
 * normalised so that sum_k w_k = 1 (the weight function carries 1/sqrt(2 pi)).
 * The roots are bracketed on a fine grid over (0, sqrt(4Q+2)] and bisected to machine
 * precision; negative roots are the mirror images, and 0 is a root when Q is odd.
 * In normalised form Q!/He_{Q+1}^2 = 1/((Q+1) h_{Q+1}^2) with h_l = He_l/sqrt(l!). */
int or_quadrature(int Q, double *p, double *w)
{
    if (Q < 1 || Q > 400) return OR_EINVAL;
    int npos = Q / 2;
    double *pos = (double *)malloc(sizeof(double) * (npos > 0 ? npos : 1));
    if (!pos) return OR_ENOMEM;
    double xmax = sqrt(4.0 * Q + 2.0) + 0.5;
    double h = 1e-3;
    int found = 0;
    double xa = 0.5 * h, fa = hermite_normalised(Q, xa);
    for (double xb = xa + h; xb <= xmax + h && found < npos; xb += h) {
        double fb = hermite_normalised(Q, xb);
        if ((fa < 0) != (fb < 0)) {
            double lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = hermite_normalised(Q, mid);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            pos[found++] = 0.5 * (lo + hi);
        }
        xa = xb;
        fa = fb;
    }
    if (found != npos) { free(pos); return OR_EROOTS; }
    int k = 0;
    for (int j = npos - 1; j >= 0; --j) p[k++] = -pos[j];
    if (Q % 2) p[k++] = 0.0;
    for (int j = 0; j < npos; ++j) p[k++] = pos[j];
    free(pos);
    for (k = 0; k < Q; ++k) {
        double hq1 = hermite_normalised(Q + 1, p[k]);
        w[k] = 1.0 / ((Q + 1) * hq1 * hq1);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------------------
 * Hermite-expanded equilibrium (Sec. II.D, eq. g_alpha):
 *   g_k[u,T] = w_k sum_{l=0}^{N} He_l(p_k) sum_{s=0}^{floor(l/2)}
 *              (T-1)^s u^(l-2s) / (2^s s! (l-2s)!)           (m = 1),
 * and f_MB^k = n g_k.  The double sum is taken literally.
 * ---------------------------------------------------------------------------------- */
void or_equilibrium(int Q, int N, const double *p, const double *w, double u, double T,
                    double *g)
{
    /* tables of j!, 2^j, (T-1)^j and u^j for j = 0..N, by repeated multiplication */
    double fact[512], two[512], tm1[512], upow[512], a[512];
    fact[0] = two[0] = tm1[0] = upow[0] = 1.0;
    for (int j = 1; j <= N; ++j) {
        fact[j] = fact[j - 1] * j;
        two[j] = two[j - 1] * 2.0;
        tm1[j] = tm1[j - 1] * (T - 1.0);
        upow[j] = upow[j - 1] * u;
    }
    for (int l = 0; l <= N; ++l) {
        double s_sum = 0.0;
        for (int s = 0; s <= l / 2; ++s)
            s_sum += tm1[s] * upow[l - 2 * s] / (two[s] * fact[s] * fact[l - 2 * s]);
        a[l] = s_sum;
    }
    for (int k = 0; k < Q; ++k) {
        /* sum_l He_l(p_k) a_l, with He_l(p_k) from the recurrence as l increases */
        double hm = 1.0, h = p[k];
        double acc = a[0];
        if (N >= 1) acc += h * a[1];
        for (int l = 1; l < N; ++l) {
            double hp = p[k] * h - l * hm;
            hm = h;
            h = hp;
            acc += h * a[l + 1];
        }
        g[k] = w[k] * acc;
    }
}

/* ------------------------------------------------------------------------------------
 * Closures (Sec. II.A-B).
 * ---------------------------------------------------------------------------------- */

/* Carnahan-Starling contact value chi_SET = (1/2)(2 - eta)/(1 - eta)^3, eta = b n / 4. */
double or_chi(double eta) { return 0.5 * (2.0 - eta) / ((1.0 - eta) * (1.0 - eta) * (1.0 - eta)); }

/* d ln chi / d ln n for chi_SET, by differentiating ln chi in eta:
 *   eta (3/(1-eta) - 1/(2-eta)) = eta (5 - 2 eta) / ((1-eta)(2-eta)).
 * Reading: the gradients are formed of {ln n, u, ln T} only (App. A.3), so
 * d_x ln chi is obtained by the chain rule from d_x ln n. */
double or_dlnchi_dlnn(double eta) { return eta * (5.0 - 2.0 * eta) / ((1.0 - eta) * (2.0 - eta)); }

/* Dense-gas Prandtl number (Sec. II.B) as a function of y = b rho chi. */
double or_prandtl_enskog(double y)
{
    double num = 1.0 + 0.8 * y + (4.0 / 25.0) * (1.0 + 12.0 / M_PI) * y * y;
    double den = 1.0 + 1.2 * y + (9.0 / 25.0) * (1.0 + 32.0 / (9.0 * M_PI)) * y * y;
    return (2.0 / 3.0) * num / den;
}

/* Relaxation time tau = mu / P_i (Sec. II.B) with the dense-gas shear viscosity
 *   mu = mu_0 b rho [1/(b rho chi) + 0.8 + (4/25)(1 + 12/pi) b rho chi],
 * mu_0 = mu_ref sqrt(T) and P_i = n T, which is
 *   tau = mu_ref (1 + 0.8 y + (4/25)(1 + 12/pi) y^2) / (n chi sqrt(T)),  y = b n chi. */
double or_tau_chi(double mu_ref, double b, double n, double T, double chi)
{
    double y = b * n * chi;
    return mu_ref * (1.0 + 0.8 * y + (4.0 / 25.0) * (1.0 + 12.0 / M_PI) * y * y) /
           (n * chi * sqrt(T));
}

double or_tau(double mu_ref, double b, double n, double T)
{
    return or_tau_chi(mu_ref, b, n, T, or_chi(0.25 * b * n));
}

/* ------------------------------------------------------------------------------------
 * Revised Enskog theory, Fischer-Methfessel prescription (Sec. II.A, eq. chi_ret): chi is
 * chi_SET of the density averaged over a ball of radius sigma.  When n depends on x only,
 * the ball's slice at offset s is a disc of area pi (sigma^2 - s^2), so
 *   nbar(x) = 3/(4 sigma^3) int_{-sigma}^{sigma} n(x + s) (sigma^2 - s^2) ds.
 * Reading: the simplified collision operator is expanded about x (Sec. II.B), so chi and
 * d ln chi are taken at the cell, d ln chi by the 6th-order central difference of ln chi
 * (App. A.3).  Between grid points n is the cubic through the four nearest points
 * (x_{m-1} .. x_{m+2} on [x_m, x_{m+1}]); outside the domain it is the periodic image, or
 * with equilibrium ghosts the end state of that side.
 * ---------------------------------------------------------------------------------- */
static double density_at(const double *n_rows, int nx, int periodic, int m)
{
    if (periodic) {
        m %= nx;
        if (m < 0) m += nx;
        return n_rows[m + OR_NG];
    }
    if (m < -OR_NG) m = -OR_NG;
    if (m > nx + OR_NG - 1) m = nx + OR_NG - 1;
    return n_rows[m + OR_NG];
}

/* nbar at cell i (any integer, ghosts included); S = sigma / dx.  Each grid interval the
 * ball covers is integrated with 4-point Gauss-Legendre, exact for the cubic times the
 * quadratic weight. */
double or_fm_density(const double *n_rows, int nx, int periodic, double S, int i)
{
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563,
                                 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461,
                                 0.6521451548625461, 0.3478548451374538};
    if (S <= 0.0) return density_at(n_rows, nx, periodic, i);
    double acc = 0.0;
    for (int m = (int)floor(-S); m < (int)ceil(S); ++m) {
        double lo = fmax((double)m, -S), hi = fmin((double)(m + 1), S);
        if (!(hi > lo)) continue;
        double f[4];
        for (int a = 0; a < 4; ++a) f[a] = density_at(n_rows, nx, periodic, i + m - 1 + a);
        for (int g = 0; g < 4; ++g) {
            double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[g];
            double x = t - m; /* position inside the interval; nodes at -1, 0, 1, 2 */
            double interp = 0.0;
            for (int a = 0; a < 4; ++a) {
                double l = 1.0;
                for (int c = 0; c < 4; ++c)
                    if (c != a) l *= (x - (c - 1)) / (double)(a - c);
                interp += l * f[a];
            }
            acc += 0.5 * (hi - lo) * gw[g] * interp * (S * S - t * t);
        }
    }
    return 0.75 / (S * S * S) * acc;
}

/* chi of every row (nx + 6 entries) from the row densities n_rows (ghost rows included;
 * with periodic boundaries only the interior rows are read). */
int or_fm_chi(const or_params *P, const double *n_rows, double *chi_rows)
{
    int R = P->nx + 2 * OR_NG;
    double S = P->sigma / P->dx;
    for (int r = 0; r < R; ++r) {
        double nb = or_fm_density(n_rows, P->nx, P->bc == OR_BC_PERIODIC, S, r - OR_NG);
        double eta = 0.25 * P->b * nb;
        if (!(nb > 0.0) || !(eta < 1.0)) return OR_EINVAL;
        chi_rows[r] = or_chi(eta);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------------------
 * Discrete moments (Sec. II.D):  n = sum phi,  n u = sum p phi,  Pxx = sum xi^2 phi,
 *   (3/2) n T = sum (xi^2 phi / 2 + theta / 2),  q = sum xi (xi^2 phi / 2 + theta / 2),
 * with xi_k = p_k - u.  Reading: the stray "d p_k" in the printed energy row is a typo.
 * ---------------------------------------------------------------------------------- */
void or_moments_row(int Q, const double *p, const double *phi, const double *theta,
                    double *n_out, double *u_out, double *T_out, double *q_out,
                    double *pxx_out)
{
    double n = 0.0, j = 0.0;
    for (int k = 0; k < Q; ++k) {
        n += phi[k];
        j += p[k] * phi[k];
    }
    double u = j / n;
    double pxx = 0.0, e = 0.0, qx = 0.0;
    for (int k = 0; k < Q; ++k) {
        double xi = p[k] - u;
        double ek = 0.5 * xi * xi * phi[k] + 0.5 * theta[k];
        pxx += xi * xi * phi[k];
        e += ek;
        qx += xi * ek;
    }
    *n_out = n;
    *u_out = u;
    *T_out = e / (1.5 * n);
    *q_out = qx;
    *pxx_out = pxx;
}

void or_moments(const or_params *P, const double *p, const double *phi, const double *theta,
                double *n, double *u, double *T, double *qx, double *pxx)
{
    int Q = P->q;
    for (int i = 0; i < P->nx; ++i) {
        int r = i + OR_NG;
        or_moments_row(Q, p, phi + (size_t)r * Q, theta + (size_t)r * Q, n + i, u + i, T + i,
                       qx + i, pxx + i);
    }
}

/* ------------------------------------------------------------------------------------
 * Sixth-order central difference (App. A.3):
 *   d_x f = [-f_{-3}/60 + 3 f_{-2}/20 - 3 f_{-1}/4 + 3 f_{+1}/4 - 3 f_{+2}/20 + f_{+3}/60] / dx.
 * `f` points at the centre value; neighbours are f[-3..3].
 * ---------------------------------------------------------------------------------- */
double or_central6(const double *f, double dx)
{
    return (-f[-3] / 60.0 + 3.0 * f[-2] / 20.0 - 3.0 * f[-1] / 4.0 + 3.0 * f[1] / 4.0 -
            3.0 * f[2] / 20.0 + f[3] / 60.0) /
           dx;
}

/* ------------------------------------------------------------------------------------
 * WENO-5 (App. A.2) for a positive advection velocity.  Given the five upwind-ordered
 * values v[0..4] = (f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2}), returns the interpolated
 * value at i+1/2 (the flux divided by the advection velocity).
 *
 * Weights: wbar_q = (delta_q / varphi_q^2) / sum_r (delta_r / varphi_r^2) with ideal
 * weights delta = (1/10, 6/10, 3/10).  When some smoothness indicators vanish exactly
 * the limiting values of Table III are used.
 * Reading: Table III is the limit in which the vanishing indicators dominate, i.e.
 * wbar_q = delta_q / sum_{r in Z} delta_r on the zero set Z and 0 elsewhere (this
 * reproduces all seven printed rows).  Otherwise the ratio is evaluated with every
 * varphi divided by the smallest one, which leaves wbar unchanged and keeps the
 * squares from underflowing when the indicators are tiny.
 * ---------------------------------------------------------------------------------- */
void or_weno_weights(const double ind[3], double wbar[3])
{
    static const double delta[3] = {0.1, 0.6, 0.3};
    int nz = 0;
    for (int q = 0; q < 3; ++q) nz += (ind[q] == 0.0);
    if (nz > 0) {
        double dz = 0.0;
        for (int q = 0; q < 3; ++q)
            if (ind[q] == 0.0) dz += delta[q];
        for (int q = 0; q < 3; ++q) wbar[q] = (ind[q] == 0.0) ? delta[q] / dz : 0.0;
        return;
    }
    double mn = ind[0];
    if (ind[1] < mn) mn = ind[1];
    if (ind[2] < mn) mn = ind[2];
    double wt[3], sum = 0.0;
    for (int q = 0; q < 3; ++q) {
        double r = mn / ind[q];
        wt[q] = delta[q] * r * r;
        sum += wt[q];
    }
    for (int q = 0; q < 3; ++q) wbar[q] = wt[q] / sum;
}

void or_weno_indicators(const double v[5], double ind[3])
{
    double a, c;
    a = v[0] - 2.0 * v[1] + v[2];
    c = v[0] - 4.0 * v[1] + 3.0 * v[2];
    ind[0] = 13.0 / 12.0 * a * a + 0.25 * c * c;
    a = v[1] - 2.0 * v[2] + v[3];
    c = v[1] - v[3];
    ind[1] = 13.0 / 12.0 * a * a + 0.25 * c * c;
    a = v[2] - 2.0 * v[3] + v[4];
    c = 3.0 * v[2] - 4.0 * v[3] + v[4];
    ind[2] = 13.0 / 12.0 * a * a + 0.25 * c * c;
}

double or_weno5(const double v[5])
{
    double f1 = v[0] / 3.0 - 7.0 * v[1] / 6.0 + 11.0 * v[2] / 6.0;
    double f2 = -v[1] / 6.0 + 5.0 * v[2] / 6.0 + v[3] / 3.0;
    double f3 = v[2] / 3.0 + 5.0 * v[3] / 6.0 - v[4] / 6.0;
    double ind[3], wb[3];
    or_weno_indicators(v, ind);
    or_weno_weights(ind, wb);
    return wb[0] * f1 + wb[1] * f2 + wb[2] * f3;
}

/* Flux of node k through interface i+1/2 given the column col[] of one distribution at
 * node k, indexed by row (cell i is row i + 3).  For p_k > 0 the stencil is
 * f_{i-2..i+2}; Reading: for p_k < 0 (not described in the paper) the stencil is the
 * mirror image f_{i+3..i-1} with the same coefficients; p_k = 0 carries no flux. */
static double interface_flux(double pk, const double *col_row_i /* row of cell i */, int Q)
{
    double v[5];
    if (pk > 0.0) {
        for (int j = 0; j < 5; ++j) v[j] = col_row_i[(j - 2) * Q];
    } else if (pk < 0.0) {
        for (int j = 0; j < 5; ++j) v[j] = col_row_i[(3 - j) * Q];
    } else {
        return 0.0;
    }
    return pk * or_weno5(v);
}

/* ------------------------------------------------------------------------------------
 * Boundary rows.  Reading: the paper does not state its boundary conditions.  Periodic
 * copies are used for the sound-wave problem; for shocks and tubes the three ghost cells
 * per side hold the equilibrium of the end state and never change.
 * ---------------------------------------------------------------------------------- */
static void fill_ghosts(const or_params *P, double *psi)
{
    if (P->bc != OR_BC_PERIODIC) return;
    int Q = P->q, nx = P->nx;
    for (int g = 0; g < OR_NG; ++g) {
        memcpy(psi + (size_t)g * Q, psi + (size_t)(nx + g) * Q, sizeof(double) * Q);
        memcpy(psi + (size_t)(nx + OR_NG + g) * Q, psi + (size_t)(OR_NG + g) * Q,
               sizeof(double) * Q);
    }
}

/* ------------------------------------------------------------------------------------
 * Per-cell sources on the lattice, for one cell with moments (n, u, T, q), Prandtl number
 * Pr, y = b n chi and gradients d ln n, d u, d ln T, d ln chi:
 *
 * Shakhov target (Sec. II.C) with f^x_MB -> n g_k (Sec. II.D), xi = p_k - u, P_i = n T:
 *   phi_S   = n g_k [1 + (1 - Pr)/(5 P_i T) (xi^2/T - 3) xi q]
 *   theta_S = 2 T n g_k [1 + (1 - Pr)/(5 P_i T) (xi^2/T - 1) xi q]
 *
 * Simplified-Enskog source (eq. j1_expanded), with f_MB -> n g_k:
 *   J1^phi   = -y [xi dlnchi + 2 xi dlnn + (3/5)(xi^2/T - 1) du
 *                 + (3/10)(xi^3/T + xi/3) dlnT] n g_k
 *   J1^theta = -y [xi dlnchi + 2 xi dlnn + (3/5)(xi^2/T - 1/3) du
 *                 + (3/10)(xi^3/T + 7 xi/3) dlnT] 2 T n g_k
 * Reading: the printed J1^phi lacks the factor b rho chi that J1^theta carries; reducing
 * the three-dimensional J1 (Sec. II.B) over p_y, p_z gives both brackets with the common
 * prefactor -b rho chi, so it is applied to both.
 * ---------------------------------------------------------------------------------- */
void or_cell_sources(int Q, int N, const double *p, const double *w, double n, double u,
                     double T, double qx, double Pr, double y, double dlnn, double du,
                     double dlnT, double dlnchi, double *phiS, double *thetaS, double *J1phi,
                     double *J1theta)
{
    double g[512];
    or_equilibrium(Q, N, p, w, u, T, g);
    double cS = (1.0 - Pr) / (5.0 * n * T * T);
    for (int k = 0; k < Q; ++k) {
        double xi = p[k] - u;
        double fk = n * g[k];
        phiS[k] = fk * (1.0 + cS * (xi * xi / T - 3.0) * xi * qx);
        thetaS[k] = 2.0 * T * fk * (1.0 + cS * (xi * xi / T - 1.0) * xi * qx);
        double bphi = xi * dlnchi + 2.0 * xi * dlnn + 0.6 * (xi * xi / T - 1.0) * du +
                      0.3 * (xi * xi * xi / T + xi / 3.0) * dlnT;
        double bth = xi * dlnchi + 2.0 * xi * dlnn + 0.6 * (xi * xi / T - 1.0 / 3.0) * du +
                     0.3 * (xi * xi * xi / T + 7.0 * xi / 3.0) * dlnT;
        J1phi[k] = -y * bphi * fk;
        J1theta[k] = -y * bth * 2.0 * T * fk;
    }
}

/* ------------------------------------------------------------------------------------
 * Right-hand side L[psi] of the discrete evolution equation (Sec. II.D and App. A.1):
 *   L_k = -(F_{i+1/2,k} - F_{i-1/2,k})/dx - (psi_k - psi_{S;k})/tau + J1_k.
 * Ghost rows of phi/theta must be filled.  Output rows cover interior cells only
 * (nx rows by q).
 * ---------------------------------------------------------------------------------- */
int or_rhs(const or_params *P, const double *p, const double *w, const double *phi,
           const double *theta, double *Lphi, double *Ltheta)
{
    int Q = P->q, nx = P->nx, N = P->nh, R = nx + 2 * OR_NG;
    double *rn = (double *)malloc(sizeof(double) * R * 5);
    if (!rn) return OR_ENOMEM;
    double *ru = rn + R, *rT = rn + 2 * R, *rq = rn + 3 * R, *rp = rn + 4 * R;
    double *lnn = (double *)malloc(sizeof(double) * R * 2);
    if (!lnn) { free(rn); return OR_ENOMEM; }
    double *lnT = lnn + R;
    double *chir = NULL, *lnchi = NULL;
    int ret = P->chi_mode == OR_CHI_RETFM;

    /* (a) moments of every row, ghosts included */
    for (int r = 0; r < R; ++r) {
        or_moments_row(Q, p, phi + (size_t)r * Q, theta + (size_t)r * Q, rn + r, ru + r, rT + r,
                       rq + r, rp + r);
        lnn[r] = log(rn[r]);
        lnT[r] = log(rT[r]);
    }
    if (ret) {
        chir = (double *)malloc(sizeof(double) * R * 2);
        if (!chir) { free(lnn); free(rn); return OR_ENOMEM; }
        lnchi = chir + R;
        int rc = or_fm_chi(P, rn, chir);
        if (rc) { free(chir); free(lnn); free(rn); return rc; }
        for (int r = 0; r < R; ++r) lnchi[r] = log(chir[r]);
    }

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        int r = i + OR_NG;
        double n = rn[r], u = ru[r], T = rT[r], qx = rq[r];
        /* (b) closures */
        double eta = 0.25 * P->b * n;
        double chi = ret ? chir[r] : or_chi(eta);
        double y = P->b * n * chi;
        double tau = or_tau_chi(P->mu_ref, P->b, n, T, chi);
        double Pr = (P->pr_mode == OR_PR_ENSKOG) ? or_prandtl_enskog(y) : P->pr;
        /* (c) gradients of ln n, u, ln T; d ln chi by the chain rule (chi_SET) or as the
         * central difference of ln chi (chi_RET-FM) */
        double dlnn = or_central6(lnn + r, P->dx);
        double du = or_central6(ru + r, P->dx);
        double dlnT = or_central6(lnT + r, P->dx);
        double dlnchi = ret ? or_central6(lnchi + r, P->dx) : or_dlnchi_dlnn(eta) * dlnn;
        /* (d)-(f) equilibrium, Shakhov target and Enskog source of every node */
        double phiS[512], thetaS[512], J1phi[512], J1th[512];
        or_cell_sources(Q, N, p, w, n, u, T, qx, Pr, y, dlnn, du, dlnT, dlnchi, phiS, thetaS,
                        J1phi, J1th);
        const double *phr = phi + (size_t)r * Q, *thr = theta + (size_t)r * Q;
        for (int k = 0; k < Q; ++k) {
            /* (g) WENO-5 fluxes through i+1/2 and i-1/2 */
            double Fp_phi = interface_flux(p[k], phr + k, Q);
            double Fm_phi = interface_flux(p[k], phr - Q + k, Q);
            double Fp_th = interface_flux(p[k], thr + k, Q);
            double Fm_th = interface_flux(p[k], thr - Q + k, Q);
            /* (h) assemble */
            Lphi[(size_t)i * Q + k] =
                -(Fp_phi - Fm_phi) / P->dx - (phr[k] - phiS[k]) / tau + J1phi[k];
            Ltheta[(size_t)i * Q + k] =
                -(Fp_th - Fm_th) / P->dx - (thr[k] - thetaS[k]) / tau + J1th[k];
        }
    }
    free(chir);
    free(lnn);
    free(rn);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------
 * Third-order TVD Runge-Kutta (App. A.1, eq. rk3 and Table II):
 *   f1 = f + dt L[f];  f2 = 3/4 f + 1/4 f1 + 1/4 dt L[f1];  f' = 1/3 f + 2/3 f2 + 2/3 dt L[f2].
 * phi/theta are (nx+6) x q arrays advanced in place by nsteps steps.
 * ---------------------------------------------------------------------------------- */
int or_step(const or_params *P, const double *p, const double *w, double *phi, double *theta,
            int nsteps)
{
    int Q = P->q, nx = P->nx, R = nx + 2 * OR_NG;
    if (Q < 1 || nx < 1 || P->nh < 0 || P->nh > Q - 1 || Q > 512) return OR_EINVAL;
    size_t full = (size_t)R * Q, inner = (size_t)nx * Q;
    double *buf = (double *)malloc(sizeof(double) * (4 * full + 2 * inner));
    if (!buf) return OR_ENOMEM;
    double *p1 = buf, *t1 = buf + full, *p2 = buf + 2 * full, *t2 = buf + 3 * full;
    double *Lp = buf + 4 * full, *Lt = Lp + inner;
    size_t off = (size_t)OR_NG * Q;
    int rc = OR_OK;
    for (int s = 0; s < nsteps && rc == OR_OK; ++s) {
        /* stage 1 */
        fill_ghosts(P, phi);
        fill_ghosts(P, theta);
        rc = or_rhs(P, p, w, phi, theta, Lp, Lt);
        if (rc) break;
        memcpy(p1, phi, sizeof(double) * full);
        memcpy(t1, theta, sizeof(double) * full);
        for (size_t j = 0; j < inner; ++j) {
            p1[off + j] = phi[off + j] + P->dt * Lp[j];
            t1[off + j] = theta[off + j] + P->dt * Lt[j];
        }
        /* stage 2 */
        fill_ghosts(P, p1);
        fill_ghosts(P, t1);
        rc = or_rhs(P, p, w, p1, t1, Lp, Lt);
        if (rc) break;
        memcpy(p2, phi, sizeof(double) * full);
        memcpy(t2, theta, sizeof(double) * full);
        for (size_t j = 0; j < inner; ++j) {
            p2[off + j] = 0.75 * phi[off + j] + 0.25 * p1[off + j] + 0.25 * P->dt * Lp[j];
            t2[off + j] = 0.75 * theta[off + j] + 0.25 * t1[off + j] + 0.25 * P->dt * Lt[j];
        }
        /* stage 3 */
        fill_ghosts(P, p2);
        fill_ghosts(P, t2);
        rc = or_rhs(P, p, w, p2, t2, Lp, Lt);
        if (rc) break;
        for (size_t j = 0; j < inner; ++j) {
            phi[off + j] = phi[off + j] / 3.0 + 2.0 * p2[off + j] / 3.0 + 2.0 * P->dt * Lp[j] / 3.0;
            theta[off + j] =
                theta[off + j] / 3.0 + 2.0 * t2[off + j] / 3.0 + 2.0 * P->dt * Lt[j] / 3.0;
        }
    }
    fill_ghosts(P, phi);
    fill_ghosts(P, theta);
    free(buf);
    return rc;
}

/* Initial state (Reading: the paper does not state it): the local equilibrium with zero
 * heat flux, phi_k = n g_k(u,T), theta_k = 2 T n g_k(u,T), for every row including the
 * ghost rows.  n,u,T have nx + 6 entries (row-indexed). */
void or_init_equilibrium(const or_params *P, const double *p, const double *w, const double *n,
                         const double *u, const double *T, double *phi, double *theta)
{
    int Q = P->q, R = P->nx + 2 * OR_NG;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
        double g[512];
        or_equilibrium(Q, P->nh, p, w, u[r], T[r], g);
        for (int k = 0; k < Q; ++k) {
            phi[(size_t)r * Q + k] = n[r] * g[k];
            theta[(size_t)r * Q + k] = 2.0 * T[r] * n[r] * g[k];
        }
    }
    fill_ghosts(P, phi);
    fill_ghosts(P, theta);
}

/* Totals of the conserved densities over the interior cells, times dx:
 *   mass sum n, momentum sum n u, energy sum (Pxx + sum theta)/2 + n u^2 / 2 ... written
 * directly as sums of the lattice moments: sum_k {phi, p phi, (p^2 phi + theta)/2}. */
void or_conserved(const or_params *P, const double *p, const double *phi, const double *theta,
                  double out[3])
{
    int Q = P->q;
    double m = 0.0, j = 0.0, e = 0.0;
    for (int i = 0; i < P->nx; ++i) {
        const double *ph = phi + (size_t)(i + OR_NG) * Q, *th = theta + (size_t)(i + OR_NG) * Q;
        for (int k = 0; k < Q; ++k) {
            m += ph[k];
            j += p[k] * ph[k];
            e += 0.5 * (p[k] * p[k] * ph[k] + th[k]);
        }
    }
    out[0] = m * P->dx;
    out[1] = j * P->dx;
    out[2] = e * P->dx;
}
