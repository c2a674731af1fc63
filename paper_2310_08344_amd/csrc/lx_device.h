// Device-side data shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime_api.h>

namespace lx {

constexpr int kKMax = 4;          // most outputs per Newton basis
constexpr int kBlockThreads = 256;

// Loop state kept in device memory.  The kernel of sweep m reads it at entry;
// the last workgroup of that sweep to finish updates it (after every other
// workgroup of the sweep has arrived), so the next sweep in the stream sees
// the new values.  The host reads it once per chunk of sweeps.
struct LejaState {
    double err[kKMax];       // last error estimate per output
    double pnorm[kKMax];     // rms norm of each output after its last update
    double ynorm;            // rms norm of the newest basis vector
    double rtol, atol;
    double fp32_switch;      // < 0: never switch to FP32 sweeps
    double scale;            // power iteration: 1 / ||w_k||
    double rho;              // power iteration: ||w_{k+1}||
    int iter;                // sweeps completed (= index m of the next sweep)
    int done;                // 1 once the loop has ended
    int status;              // lx_status
    int max_iters;
    int in32;                // y_m is stored in FP32
    int out32;               // the next sweep writes y_{m+1} in FP32
    int n_fp32;              // sweeps that wrote FP32
    int active[kKMax];       // output still iterating
    int iters[kKMax];        // sweeps until the output passed
    unsigned arrive;         // workgroups of the current sweep that finished
    int pad;
};

// Launch shape of a stencil sweep: 2-D workgroups of tx * ty threads; each
// thread owns `vec` consecutive columns and marches over `ry` rows.
struct Tile {
    int tx = 64, ty = 4, ry = 4, vec = 2;
    int cols() const { return tx * vec; }
    int rows() const { return ty * ry; }
};

struct SweepArgs {
    int nx, ny;
    int tiles_x, tiles_y;
    int K;
    int ld;                  // leading dimension of coef (per output)
    // diffusion-advection: stencil coefficients divided by gamma; aC holds
    // (c_C - c)/gamma, the sweep subtracts xi_m
    double aE, aW, aN, aS, aC;
    // Burgers Jacobian: nu/(gamma dx^2), nu/(gamma dy^2), 1/(2 gamma dx),
    // 1/(2 gamma dy), and the centre (-2 kx - 2 ky - c/gamma)
    double kx, ky, gx, gy, kC;
    double inv_sqrtN;
    const double* v;         // y_0
    void* ybuf[2];           // y_{m+1} goes to ybuf[m & 1] (FP64 or FP32)
    const double* u;         // Burgers state
    const float* u32;        // Burgers state rounded to FP32 (FP32 sweeps)
    double* p[kKMax];        // outputs (the polynomials)
    const double* base[kKMax];  // optional: p_0 = base + d_0 v (internal use)
    const double* coef;      // coef[k*ld + j] = d_j of output k
    const double* xi;        // Leja points
    double* partials;        // per-workgroup partial sums, (1+K) each
    LejaState* st;
};

struct PowerArgs {
    int nx, ny;
    int tiles_x, tiles_y;
    double cE, cW, cN, cS, cC;     // diffusion-advection stencil
    double kx, ky, gx, gy;         // Burgers: nu/dx^2, nu/dy^2, 1/(2dx), 1/(2dy)
    const double* in;
    double* out;
    const double* u;
    double* partials;
    LejaState* st;
};

enum OpCode { kOpDiffAdv = 0, kOpBurgersJ = 1 };

// Kernel launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_leja_sweep(int op, int K, bool fp32_capable, const Tile& t, const SweepArgs& a,
                             hipStream_t s);
hipError_t launch_power_sweep(int op, const Tile& t, const PowerArgs& a, hipStream_t s);
hipError_t launch_norm(const double* x, long n, double* partials, LejaState* st, hipStream_t s);
hipError_t launch_fill_splitmix(double* x, long n, unsigned long long seed, hipStream_t s);
hipError_t launch_to_fp32(const double* x, float* y, long n, hipStream_t s);
// Burgers helpers for EXPRB42
hipError_t launch_burgers_hF(const double* u, double* out, int nx, int ny, double nu, double dx,
                             double dy, double h, hipStream_t s);
hipError_t launch_burgers_remainder(const double* u, const double* U2, double* out, int nx, int ny,
                                    double nu, double dx, double dy, double h, hipStream_t s);

int num_blocks(const Tile& t, int nx, int ny);
int norm_blocks(long n);

}  // namespace lx
