// Host-side set-up arithmetic of the FDLB solver: Gauss-Hermite quadrature, the
// orthonormal Hermite table used by the equilibrium contraction, and the mapping of
// (denseness, Knudsen number) to the model's covolume and reference viscosity.
// Everything here runs once per context, in FP64, on the CPU.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace elb {

// Orthonormal probabilists' Hermite values h_l(x) = He_l(x)/sqrt(l!) for l = 0..lmax,
// from He_{l+1} = x He_l - l He_{l-1} divided through by sqrt((l+1)!).
void hermite_orthonormal(int lmax, double x, double *h)
{
    h[0] = 1.0;
    if (lmax >= 1) h[1] = x;
    for (int l = 1; l < lmax; ++l)
        h[l + 1] = (x * h[l] - std::sqrt((double)l) * h[l - 1]) / std::sqrt((double)(l + 1));
}

// Nodes: eigenvalues of the symmetric Jacobi matrix of the probabilists' Hermite
// recurrence (zero diagonal, off-diagonal sqrt(k)), found by cyclic Jacobi rotations and
// then refined by Newton's method on h_Q (h_Q' = sqrt(Q) h_{Q-1}).  Weights: Christoffel
// numbers w_k = 1 / sum_{l<Q} h_l(p_k)^2, which sum to 1 for the normalised weight
// function exp(-p^2/2)/sqrt(2 pi) of Sec. II.D.
int gauss_hermite(int Q, double *p, double *w)
{
    if (Q < 1 || Q > 256) return 1;
    std::vector<double> A((size_t)Q * Q, 0.0);
    for (int k = 1; k < Q; ++k) A[(size_t)(k - 1) * Q + k] = A[(size_t)k * Q + k - 1] = std::sqrt((double)k);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j) {
                double a = A[(size_t)i * Q + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-32 * tot) break;
        for (int r = 0; r < Q - 1; ++r)
            for (int s = r + 1; s < Q; ++s) {
                double ars = A[(size_t)r * Q + s];
                if (std::fabs(ars) < 1e-300) continue;
                double arr = A[(size_t)r * Q + r], ass = A[(size_t)s * Q + s];
                double th = (ass - arr) / (2.0 * ars);
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < Q; ++k) {  // rotate rows r, s
                    double akr = A[(size_t)r * Q + k], aks = A[(size_t)s * Q + k];
                    A[(size_t)r * Q + k] = c * akr - sn * aks;
                    A[(size_t)s * Q + k] = sn * akr + c * aks;
                }
                for (int k = 0; k < Q; ++k) {  // rotate columns r, s
                    double akr = A[(size_t)k * Q + r], aks = A[(size_t)k * Q + s];
                    A[(size_t)k * Q + r] = c * akr - sn * aks;
                    A[(size_t)k * Q + s] = sn * akr + c * aks;
                }
            }
    }
    std::vector<double> x(Q);
    for (int k = 0; k < Q; ++k) x[k] = A[(size_t)k * Q + k];
    std::sort(x.begin(), x.end());
    std::vector<double> h(Q + 2);
    for (int k = 0; k < Q; ++k) {
        for (int it = 0; it < 4; ++it) {
            hermite_orthonormal(Q, x[k], h.data());
            double d = std::sqrt((double)Q) * h[Q - 1];
            if (d == 0.0) break;
            x[k] -= h[Q] / d;
        }
    }
    // exact mirror symmetry of the node set
    for (int k = 0; k < Q / 2; ++k) {
        double a = 0.5 * (x[Q - 1 - k] - x[k]);
        x[k] = -a;
        x[Q - 1 - k] = a;
    }
    if (Q % 2) x[Q / 2] = 0.0;
    for (int k = 0; k < Q; ++k) {
        hermite_orthonormal(Q - 1, x[k], h.data());
        double s = 0.0;
        for (int l = 0; l < Q; ++l) s += h[l] * h[l];
        p[k] = x[k];
        w[k] = 1.0 / s;
    }
    return 0;
}

// Carnahan-Starling contact value (Sec. II.A, eq. chi).
double chi_set(double eta) { return 0.5 * (2.0 - eta) / ((1.0 - eta) * (1.0 - eta) * (1.0 - eta)); }

// Reduced density eta with E_l = (3/sqrt 2) b n chi = 6 sqrt(2) eta chi(eta) (Sec. II.B),
// by safeguarded Newton iteration on [0, 1/2).
double eta_of_denseness(double El)
{
    if (El <= 0.0) return 0.0;
    const double c = 6.0 * std::sqrt(2.0);
    double lo = 0.0, hi = 0.5, eta = std::min(El / c, 0.25);
    for (int it = 0; it < 200; ++it) {
        double chi = chi_set(eta);
        double f = c * eta * chi - El;
        if (f > 0) hi = eta; else lo = eta;
        double dchi = chi * (3.0 / (1.0 - eta) - 1.0 / (2.0 - eta));
        double fp = c * (chi + eta * dchi);
        double nxt = eta - f / fp;
        if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
        if (std::fabs(nxt - eta) <= 1e-17 * std::max(1.0, eta)) { eta = nxt; break; }
        eta = nxt;
    }
    return eta;
}

// Covolume b = 4 eta0 / n_ref, and the dilute hard-sphere viscosity at T = 1,
// mu_ref = (5/16) sqrt(2 pi) n_ref l_dilute, where l_dilute = chi0 * Kn * kn_length is the
// Boltzmann mean free path (the Enskog one, l = 1/(sqrt 2 pi sigma^2 n chi), divided by
// chi; Sec. II.B).  With mu_ref, tau = mu / P_i (Sec. II.B) becomes
//   tau = mu_ref (1 + 0.8 y + (4/25)(1 + 12/pi) y^2) / (n chi sqrt T),  y = b n chi.
void map_units(double El, double kn, double kn_length, double n_ref, double *b, double *mu_ref,
               double *eta0, double *chi0)
{
    double e = eta_of_denseness(El);
    double ch = chi_set(e);
    *eta0 = e;
    *chi0 = ch;
    *b = 4.0 * e / n_ref;
    *mu_ref = 5.0 / 16.0 * std::sqrt(2.0 * M_PI) * n_ref * ch * kn * kn_length;
}

// Weights of the Fischer-Methfessel ball average (Sec. II.A, eq. chi_ret) on the grid:
//   nbar_i = 3/(4 S^3) int_{-S}^{S} n(x_i + t dx) (S^2 - t^2) dt = sum_{|j|<=J} w_j n_{i+j},
// S = sigma/dx, the slice area pi (sigma^2 - s^2) of the ball being the weight in 1-D.  On
// each interval [m, m+1] (in cells) n is the cubic through the points m-1 .. m+2; w_j
// collects the exact integrals of its Lagrange basis times the weight over the part of the
// interval inside [-S, S].  Returns J (w has 2J + 1 entries, w[J] belongs to the cell).
int fm_weights(double S, std::vector<double> &w)
{
    if (!(S > 0.0)) {
        w.assign(1, 1.0);
        return 0;
    }
    const int M = (int)std::ceil(S), J = M + 1;
    w.assign(2 * J + 1, 0.0);
    for (int m = -M; m < M; ++m) {
        const double lo = std::max((double)m, -S) - m, hi = std::min((double)(m + 1), S) - m;
        if (!(hi > lo)) continue;
        // weight in x = t - m: (S^2 - m^2) - 2 m x - x^2
        const double wq[3] = {S * S - (double)m * m, -2.0 * m, -1.0};
        for (int a = 0; a < 4; ++a) {
            // Lagrange basis of node a - 1 over the nodes -1, 0, 1, 2, as coefficients in x
            double l[4] = {1.0, 0.0, 0.0, 0.0};
            double den = 1.0;
            for (int c = 0; c < 4; ++c) {
                if (c == a) continue;
                const double xc = c - 1;
                for (int d = 3; d >= 1; --d) l[d] = l[d - 1] - xc * l[d];
                l[0] = -xc * l[0];
                den *= (double)(a - c);
            }
            double integral = 0.0;
            for (int d = 0; d < 4; ++d)
                for (int e = 0; e < 3; ++e) {
                    const int k = d + e + 1;
                    integral += l[d] * wq[e] * (std::pow(hi, k) - std::pow(lo, k)) / k;
                }
            w[J + m - 1 + a] += 0.75 / (S * S * S) * integral / den;
        }
    }
    return J;
}

}  // namespace elb
