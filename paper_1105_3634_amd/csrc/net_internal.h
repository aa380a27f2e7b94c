// Hooks between the mixture (api.cpp) and the closure network (closure.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mlb.h"

namespace mlb {

// record `msg` as the calling thread's last error and return `st`
mlb_status set_error(mlb_status st, const std::string &msg);

int net_grid(const mlb_net_s *n, int *nx, int *ny, int *nz);
// changes whenever a captured inference graph of the net must be re-captured
unsigned long long net_version(const mlb_net_s *n);
// force [2][3][N] = f_ref * CNN((n_a / n_ref - 1, j_a / j_ref)) for a binary float32 state
void net_infer_fields(mlb_net_s *n, const float *dens, const float *mom, float *force, hipStream_t st);
// [6][N] float32 scratch for the closure force at check steps
float *net_check_buffer(mlb_net_s *n);
double *net_err_buffer(mlb_net_s *n, int *nparts);
// training pair from a state and its exact force: x_out [8][N], target_out [6][N] (float32)
void net_sample(mlb_net_s *n, const float *dens, const float *mom, const float *force, float *x_out,
                float *target_out, hipStream_t st);

}  // namespace mlb
