// Host-side set-up arithmetic (quadrature, Hermite table, unit mapping).
#pragma once

#include <vector>

namespace elb {

void hermite_orthonormal(int lmax, double x, double *h);
int gauss_hermite(int Q, double *p, double *w);
double chi_set(double eta);
double eta_of_denseness(double El);
void map_units(double El, double kn, double kn_length, double n_ref, double *b, double *mu_ref,
               double *eta0, double *chi0);
int fm_weights(double S, std::vector<double> &w);

}  // namespace elb
