// Shapes, layouts and launchers of the predictor MLP (8 -> 64 -> 64 -> 2).
#pragma once

#include <hip/hip_runtime_api.h>

namespace lx {

constexpr int kMlpIn = 8, kMlpH = 64, kMlpOut = 2;

// parameter vector: W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]
constexpr int kPW1 = 0;
constexpr int kPB1 = kPW1 + kMlpH * kMlpIn;
constexpr int kPW2 = kPB1 + kMlpH;
constexpr int kPB2 = kPW2 + kMlpH * kMlpH;
constexpr int kPW3 = kPB2 + kMlpH;
constexpr int kPB3 = kPW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kPB3 + kMlpOut;   // 4866

// per-sample scratch row of a training step
constexpr int kOffX = 0;
constexpr int kOffA1 = kOffX + kMlpIn;
constexpr int kOffA2 = kOffA1 + kMlpH;
constexpr int kOffDz1 = kOffA2 + kMlpH;
constexpr int kOffDz2 = kOffDz1 + kMlpH;
constexpr int kOffDy = kOffDz2 + kMlpH;
constexpr int kOffLoss = kOffDy + kMlpOut;
constexpr int kMlpRow = kOffLoss + 2;

// standardisation of inputs and targets (passed by value to the kernels)
struct MlpScaling {
    float mean_x[kMlpIn], std_x[kMlpIn];
    float mean_y[kMlpOut], std_y[kMlpOut];
};

struct FeatureInst {
    int nx, ny, l, burgers;
    double dx, h, D, vx, vy;   // D holds nu for Burgers
    const double* u;           // the Burgers state, else the input vector
};

hipError_t launch_mlp_fwd_bwd(const float* theta, const float* X, const float* Y, const int* idx, int B,
                              const MlpScaling& sc, float* scratch, hipStream_t s);
hipError_t launch_mlp_grad(const float* scratch, int B, float* grad, double* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr, hipStream_t s);
hipError_t launch_mlp_infer(const float* theta, const float* X, int n, const MlpScaling& sc, float* Y,
                            hipStream_t s);
hipError_t launch_features(const FeatureInst* fi, int n, float* X, hipStream_t s);

}  // namespace lx
