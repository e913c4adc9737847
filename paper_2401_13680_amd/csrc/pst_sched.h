// Host-only definition of the run-time model (pst_model of include/pst.h),
// shared by the scheduling functions and the request server.
#pragma once
#include <vector>

struct pst_model {
    int degree;
    std::vector<double> u, w, v, ms;   // observations (scaled sizes) and run times
    std::vector<double> coef;          // one per monomial, graded order
    bool fitted = false;
};
