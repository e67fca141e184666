// Probe-count predictor (a small multilayer perceptron) shared between the
// network's own entry points and the IVFADC search that uses it.
#pragma once

#include "common.hpp"

struct mk_mlp;

namespace mk {

// Number of raw features the predictor of an index with d dimensions reads:
// the query and its 32 smallest squared coarse distances.
constexpr int kProbeDists = 32;

int32_t mlp_inputs(const mk_mlp* net);

// yhat[i] = network(standardised F[i]) for n rows of mlp_inputs() floats.
mk_status mlp_forward_dev(const mk_mlp* net, const float* F, int64_t n, float* yhat,
                          hipStream_t s);

}  // namespace mk
