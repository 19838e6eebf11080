// Launchers of the learned surrogate's kernels (features, plain estimate,
// targets, choice, and the network's layers), defined next to their kernels.
// All return hipError_t of the launch.
#pragma once

#include "rt_internal.h"

namespace rc {

hipError_t launch_features(const Geo& g, const uint32_t* band_hist, const uint32_t* whole_hist, float* X,
                           hipStream_t st);
hipError_t launch_estimate_new(const Geo& g, const uint64_t* band_sums, double* p_new, int32_t* status,
                               hipStream_t st);
hipError_t launch_targets(const Geo& g, const double* p_new, const int32_t* status, float* T, uint8_t* mask,
                          hipStream_t st);
hipError_t launch_features_new(const Geo& g, const uint32_t* band_hist, const uint64_t* band_sums,
                               const uint32_t* whole_hist, float* X, double* p_new, int32_t* status, hipStream_t st);
hipError_t launch_select_lut(const Geo& g, const float* H2, const float* W3, const float* b3, float* Y,
                             const double* p_new, const int32_t* status, float tol, const Bufs& b, uint8_t* used,
                             float* residual, hipStream_t st);
hipError_t launch_select(const Geo& g, const float* Y, const double* p_new, const int32_t* status, float tol,
                         double* params, uint8_t* valid, uint8_t* used, float* residual, hipStream_t st);
// The two hidden layers only (H1, H2); the output layer is then
// wave_row_dot per row, as in mlp_forward.
hipError_t mlp_hidden(const float* const* w, const float* X, int n, float* H1, float* H2, hipStream_t st);
// With T, the output layer also writes the loss gradient dY (training).
hipError_t mlp_forward(const float* const* w, const float* X, int n, float* H1, float* H2, float* Y, hipStream_t st,
                       const float* T = nullptr, float* dY = nullptr);
hipError_t mlp_backward(const float* const* w, const float* X, const float* H1, const float* H2, const float* Y,
                        const float* T, int n, float* const* g, float* dY, float* dZ1, float* dZ2, hipStream_t st,
                        bool dy_ready = false);   // dy_ready: dY already holds the loss gradient
hipError_t mlp_adam(float* const* w, const float* const* g, float* const* m, float* const* v, int step, float lr,
                    float beta1, float beta2, float eps, hipStream_t st);
hipError_t mlp_mse(const float* Y, const float* T, int n, float* out, hipStream_t st);
hipError_t gather_rows(const float* src, int row_len, const int32_t* idx, int n, float* dst, hipStream_t st);
hipError_t gather_rows2(const float* a, int la, float* da, const float* b, int lb, float* db, const int32_t* idx, int n,
                       hipStream_t st);

}  // namespace rc
