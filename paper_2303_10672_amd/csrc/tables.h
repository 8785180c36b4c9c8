// Host table builders (FP64).
#pragma once

#include <string>
#include <vector>

#include "pvi.h"

namespace pvi {

double gamma_p(double a, double x);
double gamma_q(double a, double x);
double binom_pmf(int k, int n, double rho);

// One demand PMF row over 0..dmax with the tail folded into dmax.
bool demand_row(int kind, double mean, double shape, int dmax, const double* table,
                std::vector<double>& out, std::string& err);

}  // namespace pvi
