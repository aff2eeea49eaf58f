// lbm_host.h - host-side model queries used by the C-ABI layer.
#pragma once

#include <cstdint>
#include <string>

#include "lbm_model.h"

namespace lbm {

bool model_from_shape(int D, int Q, ModelId& m);
int model_dim(ModelId m);
int model_q(ModelId m);
int model_groups(ModelId m);
int model_group_of(ModelId m, int i);
int model_e(ModelId m, int i, int k);
int model_e2(ModelId m, int g);
// True if e (int32[Q][D]) is the canonical velocity list of the model.
bool model_matches(ModelId m, const int32_t* e);
// Largest absolute residual of Formula (5) at group weights W and speed c.
double model_residual(ModelId m, const double* W, double c);
// Newton solution of Formula (5) for the group weights and c.
bool model_solve(ModelId m, double* W, double* c, std::string& err);

}  // namespace lbm
