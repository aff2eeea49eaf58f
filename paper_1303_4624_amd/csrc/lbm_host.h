// lbm_host.h - host-side model queries used by the C-ABI layer.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "lbm_model.h"

namespace lbm {

bool model_from_shape(int D, int Q, ModelId& m);
int model_dim(ModelId m);
int model_q(ModelId m);
int model_groups(ModelId m);
int model_group_of(ModelId m, int i);
int model_e(ModelId m, int i, int k);
int model_e2(ModelId m, int g);
// Order of accuracy m of a compiled model (its equilibrium has order N = m).
int model_order(ModelId m);
// True if e (int32[Q][D]) is the canonical velocity list of the model.
bool model_matches(ModelId m, const int32_t* e);
// Largest absolute residual of Formula (5) at group weights W and speed c.
double model_residual(ModelId m, const double* W, double c);
// Newton solution of Formula (5) for the group weights and c.
bool model_solve(ModelId m, double* W, double* c, std::string& err);

// Number of equations of Formula (5) up to order 2m in D dimensions
// (Omega(m, D) of Formula (8)).
int equation_count(int m, int D);

// A model built from arbitrary group representatives.
struct BuiltModel {
    int D = 0, Q = 0, G = 0;
    std::vector<std::array<int, 3>> e;
    std::vector<int> group;
    std::vector<double> W;
    double c = 0, residual = 0;
};
// Orbits of reps (int32[G][D]) and the Newton solution of Formula (5) up to
// order 2m from the given guesses (w_guess may be NULL: least squares at
// c_guess).  Fails unless G + 1 = Omega(m, D) (Formula (10)).
bool model_build(int D, int m, int G, const int32_t* reps, const double* w_guess, double c_guess,
                 BuiltModel& out, std::string& err);

}  // namespace lbm
