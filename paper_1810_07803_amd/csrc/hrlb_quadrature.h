// hrlb_quadrature.h -- extended-precision recurrences and Gauss rules (host only).
#pragma once
#include <vector>

namespace hrlb {

struct Recurrence {
    std::vector<long double> alpha, beta;  // monic: p_{k+1} = (z - alpha_k) p_k - beta_k p_{k-1}; beta_0 = mass
};

Recurrence half_range_recurrence(int n);
Recurrence hermite_recurrence(int n);
void orthonormal_values(const Recurrence& r, int L, long double z, long double* out);
void gauss_from_recurrence(const Recurrence& r, int n, std::vector<long double>& nodes,
                           std::vector<long double>& weights);

}  // namespace hrlb
