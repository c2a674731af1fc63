// HIP kernels (gfx950) of the spectral/budget predictor: an MLP
// 8 -> 64 -> 64 -> 2 with ReLU, float32 weights and bfloat16 hidden
// activations, trained with Adam on the mean squared error.
//
// Training step on a minibatch of B samples:
//   mlp_fwd_bwd_kernel  one thread per sample: standardise, forward, loss,
//                       backward to the per-sample deltas (float32); writes
//                       the sample's inputs, activations and deltas
//   mlp_grad_kernel     one thread per parameter: sums its gradient over the
//                       minibatch in sample order (float64 accumulation)
//   mlp_adam_kernel     one thread per parameter
// The network is tiny (4866 parameters, ~4.7k multiply-adds per sample):
// the kernels are latency-bound, and the fixed summation order makes every
// step deterministic.
#include <hip/hip_runtime.h>

#include "mlp_device.h"

namespace lx {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ float to_bf16(float x) {
    // round to nearest even on the upper 16 bits of the float32 pattern
    unsigned u = __float_as_uint(x);
    const unsigned lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    return __uint_as_float(u);
}

struct Net {
    const float* W1;
    const float* b1;
    const float* W2;
    const float* b2;
    const float* W3;
    const float* b3;
};

__device__ __forceinline__ Net net_of(const float* theta) {
    Net n;
    n.W1 = theta;
    n.b1 = n.W1 + kMlpH * kMlpIn;
    n.W2 = n.b1 + kMlpH;
    n.b2 = n.W2 + kMlpH * kMlpH;
    n.W3 = n.b2 + kMlpH;
    n.b3 = n.W3 + kMlpOut * kMlpH;
    return n;
}

// forward of one standardised sample; a1, a2 rounded to bfloat16, z masks kept
__device__ __forceinline__ void forward_one(const Net& n, const float (&x)[kMlpIn], float (&a1)[kMlpH],
                                            float (&a2)[kMlpH], float (&y)[kMlpOut]) {
    for (int i = 0; i < kMlpH; ++i) {
        float z = n.b1[i];
#pragma unroll
        for (int j = 0; j < kMlpIn; ++j) z = fmaf(n.W1[i * kMlpIn + j], x[j], z);
        a1[i] = to_bf16(fmaxf(z, 0.0f));
    }
    for (int i = 0; i < kMlpH; ++i) {
        float z = n.b2[i];
        for (int j = 0; j < kMlpH; ++j) z = fmaf(n.W2[i * kMlpH + j], a1[j], z);
        a2[i] = to_bf16(fmaxf(z, 0.0f));
    }
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        float z = n.b3[o];
        for (int j = 0; j < kMlpH; ++j) z = fmaf(n.W3[o * kMlpH + j], a2[j], z);
        y[o] = z;
    }
}

__global__ __launch_bounds__(kT) void mlp_fwd_bwd_kernel(const float* __restrict__ theta,
                                                         const float* __restrict__ X, const float* __restrict__ Y,
                                                         const int* __restrict__ idx, int B, MlpScaling sc,
                                                         float* __restrict__ scratch) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const Net n = net_of(theta);
    const int r = idx ? idx[s] : s;
    float x[kMlpIn], t[kMlpOut];
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) x[j] = (X[static_cast<long>(r) * kMlpIn + j] - sc.mean_x[j]) / sc.std_x[j];
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) t[o] = (Y[static_cast<long>(r) * kMlpOut + o] - sc.mean_y[o]) / sc.std_y[o];
    float a1[kMlpH], a2[kMlpH], y[kMlpOut];
    forward_one(n, x, a1, a2, y);
    float* __restrict__ row = scratch + static_cast<long>(s) * kMlpRow;
    float dY[kMlpOut];
    float loss = 0.0f;
    const float scale = 2.0f / static_cast<float>(B * kMlpOut);
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        const float d = y[o] - t[o];
        loss = fmaf(d, d, loss);
        dY[o] = scale * d;
    }
    // dz2 = (W3^T dY) * [a2 > 0]   (a2 > 0 exactly when z2 > 0)
    float dz2[kMlpH];
    for (int j = 0; j < kMlpH; ++j) {
        float g = 0.0f;
#pragma unroll
        for (int o = 0; o < kMlpOut; ++o) g = fmaf(n.W3[o * kMlpH + j], dY[o], g);
        dz2[j] = a2[j] > 0.0f ? g : 0.0f;
    }
    // dz1 = (W2^T dz2) * [a1 > 0]
    for (int j = 0; j < kMlpH; ++j) {
        float g = 0.0f;
        for (int i = 0; i < kMlpH; ++i) g = fmaf(n.W2[i * kMlpH + j], dz2[i], g);
        row[kOffDz1 + j] = a1[j] > 0.0f ? g : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) row[kOffX + j] = x[j];
    for (int j = 0; j < kMlpH; ++j) {
        row[kOffA1 + j] = a1[j];
        row[kOffA2 + j] = a2[j];
        row[kOffDz2 + j] = dz2[j];
    }
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) row[kOffDy + o] = dY[o];
    row[kOffLoss] = loss;
}

// gradient of parameter p summed over the minibatch in sample order
__global__ __launch_bounds__(kT) void mlp_grad_kernel(const float* __restrict__ scratch, int B,
                                                      float* __restrict__ grad, double* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out != nullptr) {
        double L = 0.0;
        for (int s = 0; s < B; ++s) L += scratch[static_cast<long>(s) * kMlpRow + kOffLoss];
        *loss_out = L / (static_cast<double>(B) * kMlpOut);
    }
    if (p >= kMlpParams) return;
    int off_a, off_b;   // gradient = sum_s row[off_a] * row[off_b] (off_b < 0: bias)
    if (p < kPW1 + kMlpH * kMlpIn) {
        const int q = p - kPW1;
        off_a = kOffDz1 + q / kMlpIn;
        off_b = kOffX + q % kMlpIn;
    } else if (p < kPB1 + kMlpH) {
        off_a = kOffDz1 + (p - kPB1);
        off_b = -1;
    } else if (p < kPW2 + kMlpH * kMlpH) {
        const int q = p - kPW2;
        off_a = kOffDz2 + q / kMlpH;
        off_b = kOffA1 + q % kMlpH;
    } else if (p < kPB2 + kMlpH) {
        off_a = kOffDz2 + (p - kPB2);
        off_b = -1;
    } else if (p < kPW3 + kMlpOut * kMlpH) {
        const int q = p - kPW3;
        off_a = kOffDy + q / kMlpH;
        off_b = kOffA2 + q % kMlpH;
    } else {
        off_a = kOffDy + (p - kPB3);
        off_b = -1;
    }
    double acc = 0.0;
    for (int s = 0; s < B; ++s) {
        const float* row = scratch + static_cast<long>(s) * kMlpRow;
        const double a = row[off_a];
        acc += off_b >= 0 ? a * static_cast<double>(row[off_b]) : a;
    }
    grad[p] = static_cast<float>(acc);
}

__global__ __launch_bounds__(kT) void mlp_adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                      float* __restrict__ m, float* __restrict__ v, int t, float lr,
                                                      float beta1, float beta2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mhat = mm / (1.0f - powf(beta1, static_cast<float>(t)));
    const float vhat = vv / (1.0f - powf(beta2, static_cast<float>(t)));
    theta[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

__global__ __launch_bounds__(kT) void mlp_infer_kernel(const float* __restrict__ theta, const float* __restrict__ X,
                                                       int n, MlpScaling sc, float* __restrict__ Yout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const Net net = net_of(theta);
    float x[kMlpIn];
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) x[j] = (X[static_cast<long>(s) * kMlpIn + j] - sc.mean_x[j]) / sc.std_x[j];
    float a1[kMlpH], a2[kMlpH], y[kMlpOut];
    forward_one(net, x, a1, a2, y);
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) Yout[static_cast<long>(s) * kMlpOut + o] = y[o] * sc.std_y[o] + sc.mean_y[o];
}

// features of one instance per workgroup: log D, log(|v| + 1e-3), angle,
// log dx, log h, log rms(u), log max|u|, l (Burgers: D := nu,
// |v| := sqrt(2) max|u|, angle := pi/4; u is the Burgers state, else v)
__global__ __launch_bounds__(kT) void features_kernel(const FeatureInst* __restrict__ fi, float* __restrict__ X) {
    const FeatureInst& f = fi[blockIdx.x];
    const long N = static_cast<long>(f.nx) * f.ny;
    double ss = 0.0, mx = 0.0;
    for (long t = threadIdx.x; t < N; t += blockDim.x) {
        const double q = f.u[t];
        ss += q * q;
        mx = fmax(mx, fabs(q));
    }
    __shared__ double red_s[kT], red_m[kT];
    red_s[threadIdx.x] = ss;
    red_m[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            red_s[threadIdx.x] += red_s[threadIdx.x + w];
            red_m[threadIdx.x] = fmax(red_m[threadIdx.x], red_m[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rms = sqrt(red_s[0] / static_cast<double>(N));
        const double umax = red_m[0];
        float* x = X + static_cast<long>(blockIdx.x) * kMlpIn;
        if (f.burgers) {
            x[0] = static_cast<float>(log(f.D));
            x[1] = static_cast<float>(log(sqrt(2.0) * umax + 1e-3));
            x[2] = static_cast<float>(0.7853981633974483);
        } else {
            x[0] = static_cast<float>(log(f.D));
            x[1] = static_cast<float>(log(sqrt(f.vx * f.vx + f.vy * f.vy) + 1e-3));
            x[2] = static_cast<float>(atan2(f.vy, f.vx));
        }
        x[3] = static_cast<float>(log(f.dx));
        x[4] = static_cast<float>(log(f.h));
        x[5] = static_cast<float>(log(rms + 1e-300));
        x[6] = static_cast<float>(log(umax + 1e-300));
        x[7] = static_cast<float>(f.l);
    }
}

}  // namespace

hipError_t launch_mlp_fwd_bwd(const float* theta, const float* X, const float* Y, const int* idx, int B,
                              const MlpScaling& sc, float* scratch, hipStream_t s) {
    hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3((B + kT - 1) / kT), dim3(kT), 0, s, theta, X, Y, idx, B, sc, scratch);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* scratch, int B, float* grad, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((kMlpParams + kT - 1) / kT), dim3(kT), 0, s, scratch, B, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + kT - 1) / kT), dim3(kT), 0, s, theta, grad, m, v, t, lr,
                       0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* theta, const float* X, int n, const MlpScaling& sc, float* Y,
                            hipStream_t s) {
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((n + kT - 1) / kT), dim3(kT), 0, s, theta, X, n, sc, Y);
    return hipGetLastError();
}

hipError_t launch_features(const FeatureInst* fi, int n, float* X, hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(n), dim3(kT), 0, s, fi, X);
    return hipGetLastError();
}

}  // namespace lx
