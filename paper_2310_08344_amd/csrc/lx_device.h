// Device-side data shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime_api.h>

namespace lx {

constexpr int kKMax = 4;          // most outputs per Newton basis
constexpr int kBlockThreads = 256;

// State of the Newton-Leja loop as it enters one sweep.
struct SweepState {
    double err[kKMax];       // last error estimate per output
    double pnorm[kKMax];     // rms norm of each output after its last update
    double ynorm;            // rms norm of the newest basis vector
    int active[kKMax];       // output still iterating during this sweep
    int iters[kKMax];        // sweeps until the output passed the test
    int in32;                // y_m is stored in FP32
    int out32;               // this sweep writes y_{m+1} in FP32
    int n_fp32;              // sweeps so far that wrote FP32
    int status;              // lx_status
    int done;                // the loop has ended
    int iter;                // sweeps completed (leja_block: the window's first term index m)
    // leja_block (several iterations per launch, speculative windows):
    int blk_mode;            // 0: a window whose terms are added speculatively; 1: its re-execution
    int nt[kKMax];           // terms each output takes in this launch (0..depth; -j: stops after j)
    int n_work;              // launches that did work so far
    int n_levels;            // operator applications they made
    double bytes_pp;         // their algorithmic bytes per grid point
};

// Loop control in device memory.  There is no synchronisation between the
// workgroups of one sweep: sweep m writes per-workgroup partial sums into
// partials[m & 1]; every workgroup of sweep m+1 adds all of them in the same
// fixed order, so all reach the same stop decision, and workgroup 0 records
// it in slot[(m+1) & 1].  Kernel boundaries make each sweep's writes visible
// to the next.  slot[2] receives the final state once the loop ends; later
// sweeps see its done flag and return at once.
struct LoopCtl {
    SweepState slot[3];
    double rtol, atol;
    double fp32_switch;      // < 0: never switch to FP32 sweeps
    double rho;              // power iteration result
    int max_iters;
    int pad;
};

// Launch shape of a stencil sweep: 2-D workgroups of tx * ty threads; each
// thread owns `vec` consecutive columns and marches over `ry` rows; `nb`
// workgroups (0 = one per tile) loop over the tiles.
struct Tile {
    int tx = 64, ty = 4, ry = 4, vec = 2, nb = 0;
    int depth = 1;           // Leja iterations per launch: 1 (leja_sweep), 2 (leja_pair), 3+ (windows)
    int th = 16;             // tile rows of leja_pair and leja_block (their tiles are 128 columns wide)
    int pnb = 1024;          // workgroups of leja_pair and leja_block
    int stream = 0;          // windows by register streaming (leja_stream) instead of LDS tiles
    int bands = 0;           // leja_stream: bands of rows (0: one resident round of wavefronts)
    int snb = 0;             // leja_stream: workgroups (0: as many as hold the items, up to one round)
    int cols() const { return tx * vec; }
    int rows() const { return ty * ry; }
};

// Static device scratch of lx_phi_leja_static (static_ws.hip): the basis
// pair and the windows' second output buffers for grids of at most
// kStaticPoints points, then kStaticPartials partial sums.
constexpr size_t kStaticPoints = size_t{1} << 18;
constexpr size_t kStaticPartials = size_t{2} * 4096 * 8 * (1 + kKMax);
constexpr size_t kStaticDoubles = (2 + kKMax) * kStaticPoints + kStaticPartials;
// The scratch's address on `device` (looked up once per device).
hipError_t static_scratch(int device, double** out);

// Launch shape of a batch, chosen by lx_tune_batched per batch class: Leja
// iterations per launch (1, 2 or kBatchBlockDepth), tile rows of the two-
// iteration and window kernels, and the points each workgroup of an
// instance serves.  Zero fields take the default rule.
struct BatchShape {
    int depth = 0, th = 0, ppw = 0;
};

struct SweepArgs {
    int nx, ny;
    int tiles_x, tiles_y;
    int nb;                  // workgroups in the grid (every sweep uses the same)
    int ld;                  // leading dimension of coef (per output)
    // diffusion-advection: stencil coefficients divided by gamma; aC holds
    // (c_C - c)/gamma, the sweep subtracts xi_m
    double aE, aW, aN, aS, aC;
    // third-order upwind advection: the second neighbours (one of each pair is 0)
    double aE2, aW2, aN2, aS2;
    // Burgers Jacobian: nu/(gamma dx^2), nu/(gamma dy^2), 1/(2 gamma dx),
    // 1/(2 gamma dy), and the centre (-2 kx - 2 ky - c/gamma)
    double kx, ky, gx, gy, kC;
    double inv_sqrtN;
    const double* v;         // y_0
    void* ybuf[2];           // y_{m+1} goes to ybuf[m & 1] (FP64 or FP32)
    const double* u;         // Burgers state
    const float* u32;        // Burgers state rounded to FP32 (FP32 sweeps)
    double* p[kKMax];        // outputs (the polynomials)
    double* p2[kKMax];       // leja_block: second buffer of each output (windows alternate)
    const double* coef;      // coef[k*ld + j] = d_j of output k
    const double* xi;        // Leja points
    double* partials;        // [2][nb][1+K]
    LoopCtl* ctl;
    SweepState* pub;         // host-visible copy of the final state (pinned host memory), or NULL
};

struct PowerArgs {
    int nx, ny;
    int tiles_x, tiles_y;
    int nb;
    double cE, cW, cN, cS, cC;     // diffusion-advection stencil
    double cE2, cW2, cN2, cS2;     // its second neighbours (third-order upwind)
    double kx, ky, gx, gy;         // Burgers: nu/dx^2, nu/dy^2, 1/(2dx), 1/(2dy)
    const double* in;
    double* out;
    const double* u;
    const double* add;             // rhs_sweep: the source S (else NULL)
    double* partials;              // [2][nb]
    LoopCtl* ctl;
};

// kOpDiffAdv3: diffusion with third-order upwind advection, a radius-2 cross
// stencil (the others have radius 1)
enum OpCode { kOpDiffAdv = 0, kOpBurgersJ = 1, kOpDiffAdv3 = 2 };

// One instance of a batch: its operator, vectors and its share of the
// workgroups of every batched launch.  c, gamma and rho are written by the
// batched power iteration when it runs.
struct BatchInst {
    int kind;                // OpCode
    int nx, ny;
    int vec;                 // columns per lane (2 when nx is even and rows are 16-byte aligned)
    int l;                   // phi order
    int tiles_x, tiles_y;    // tiles of the Leja kernel in use (one- or two-iteration layout)
    int ptiles_x, ptiles_y;  // tiles of the power-iteration sweeps (kBatchTx * vec x kBatchTy * kBatchPowerRows)
    int wg_begin, nb;        // workgroups [wg_begin, wg_begin + nb) of each launch
    int has_x0;              // x0 given; else a splitmix64 vector in y[1]
    long part_off;           // offset of its partial sums: [2][nb][2]
    double dx, dy, D, vx, vy, nu;
    double h, c, gamma, rho;
    double pw[5];            // stencil of A (power iteration), from the host
    double st[5];            // stencil of (A - c)/gamma (Leja sweeps), host or batched power iteration
    const double* u;
    const double* v;
    double* out;
    double* out2;            // second output buffer (windows), else NULL
    const double* x0;
    double* y[2];            // basis (and power iteration) buffers
};

constexpr int kBatchTx = 32, kBatchTy = 8;   // workgroup shape of the batched sweeps
constexpr int kBatchPowerRows = 4;           // rows each thread of a batched power sweep marches over

// Kernel launchers (kernels.hip).  Each returns the hipError_t of the launch.
// Sweep m of the Leja loop (m = max_iters only takes the last decision).
hipError_t launch_leja_sweep(int op, int K, bool fp32_capable, const Tile& t, const SweepArgs& a, int m,
                             hipStream_t s);
// Launch L of the two-iterations-per-launch loop (pair.hip): sweeps 2L and
// 2L+1 on tiles of 128 x th points (th in {8, 16, 32}); FP64, nx even.
hipError_t launch_leja_pair(int op, int K, int th, const SweepArgs& a, int L, hipStream_t s);
// Launch L of the loop with `depth` (3, 4 or 6) iterations per launch
// (block.hip): speculative windows re-executed when an output stops inside
// one; tiles of 128 x th points (th in {8, 16}); FP64, nx even, sides of at
// least depth x radius cells; every operator at depths 3 and 4 (Burgers
// needs a.u), the five-point diffusion-advection operator also at 6.
hipError_t launch_leja_block(int op, int K, int th, int depth, const SweepArgs& a, int L, hipStream_t s);
// Power iteration: norm of the start vector into partials[1], then sweeps
// k = 0..iters-1, then the final norm into ctl->rho.
hipError_t launch_power_norm(const double* x, long n, int nb, double* partials, hipStream_t s);
hipError_t launch_power_sweep(int op, const Tile& t, const PowerArgs& a, int k, hipStream_t s);
hipError_t launch_power_final(int nb, const double* partials, LoopCtl* ctl, hipStream_t s);
// Power iteration with kPowerBlockDepth sweeps per launch (block.hip; every
// operator (Burgers needs a.u), nx even, 128-column tiles of
// power_block_rows(op) rows with a.tiles_x/a.tiles_y in that layout): launch b makes nlev (1..depth)
// levels from `in`; the start vector's norm partials at partials[nb + i]
// (launch_power_norm), its own at partials[2 nb + (b & 1) nb depth + ...];
// partials needs 2 nb (1 + depth) doubles.  Then the final ratio into
// ctl->rho.
constexpr int kPowerBlockDepth = 4;
// op: kOpDiffAdv (tiles of 128 x 16), kOpDiffAdv3 or kOpBurgersJ (128 x 8)
int power_block_rows(int op);
// workgroups of power_block that are resident at once on the current device
// (0 if the runtime cannot tell)
int power_block_resident(int op);
hipError_t launch_power_block(int op, const PowerArgs& a, const double* in, double* out, int b, int nlev,
                              hipStream_t s);
hipError_t launch_power_block_final(const PowerArgs& a, int b, int nlev, hipStream_t s);
// Windows by register streaming (stream.hip; the five-point
// diffusion-advection operator or the Burgers Jacobian (a.u, and a.u32 for
// FP32 sweeps), nx even, sides >= depth, 16-byte aligned vectors); fp32:
// FP32 sweeps (the device switches windows to FP32 levels, LoopCtl
// fp32_switch); a.tiles_x = stream_strips(nx, depth) strips of at most
// 128 - 2 depth output columns (edges on 128-byte lines where that costs at
// most four of them) by a.tiles_y (1..ny) bands of rows, a.nb
// workgroups of four wavefronts that each take items (strip, band) in turn;
// partials as launch_leja_block.
int stream_strips(int nx, int depth);
// whether leja_stream is built for this operator (kOp*), K outputs, depth
// and precision mode
bool stream_has(int op, int K, int depth, bool fp32);
hipError_t launch_leja_stream(int op, int K, int depth, bool fp32, const SweepArgs& a, int L, hipStream_t s);
// workgroups of that leja_stream (power = 0) or of power_stream (power = 1)
// resident at once on the current device (0 if unknown)
int stream_resident(int op, int K, int depth, bool fp32, int power);
// Power iteration by register streaming, up to kPowerStreamDepth sweeps per
// launch (the five-point diffusion-advection operator; nx even, sides >=
// kPowerStreamDepth, a.tiles_x = stream_strips(nx, kPowerStreamDepth),
// a.tiles_y bands); partials need 2 nb (1 + kPowerStreamDepth) doubles, laid
// out as for launch_power_block with kPowerStreamDepth in place of its depth.
constexpr int kPowerStreamDepth = 10;
// Launch b makes nlev levels, scaled by the norm of the prev levels of
// launch b - 1 (of the start vector for b = 0, from launch_power_norm).
// raw0: launch 0 takes the start vector unscaled (nlev = kPowerStreamDepth)
// and records its norm in place of launch_power_norm; the final launch then
// gives a NaN estimate unless ||x||^2 lay in [1e-200, 1e20] (the host then
// repeats the iteration with the norm first).
hipError_t launch_power_stream(const PowerArgs& a, const double* in, double* out, int b, int nlev, int prev,
                               bool raw0, hipStream_t s);
hipError_t launch_power_stream_final(const PowerArgs& a, int b, int nlev, bool raw0, hipStream_t s);
hipError_t launch_fill_splitmix(double* x, long n, unsigned long long seed, hipStream_t s);
hipError_t launch_to_fp32(const double* x, float* y, long n, hipStream_t s);
// kind 0: z = x (copy); kind 1: z = 1.5 x - 0.5 y.  n even.
hipError_t launch_probe(int kind, const double* x, const double* y, double* z, long n, hipStream_t s);
// Burgers helpers for EXPRB42
hipError_t launch_burgers_hF(const double* u, double* out, int nx, int ny, double nu, double dx,
                             double dy, double h, hipStream_t s);
// h [N(u + a) - N(u)], N(w) = F(w) - J(u) w
hipError_t launch_burgers_remainder(const double* u, const double* a, double* out, int nx, int ny,
                                    double nu, double dx, double dy, double h, hipStream_t s);
// out = h (A u + S) with a tiled sweep (PowerArgs: stencil of A, in = u,
// out, add = S or NULL; the shape of lx_spectrum's power sweeps)
hipError_t launch_rhs_sweep(int op, const Tile& t, const PowerArgs& a, double h, hipStream_t s);
// out = b * base + sum_i a[i] * x[i] (base may be NULL; at most 8 terms)
struct LinComb {
    const double* x[8];
    double a[8];
    int n_terms;
};
hipError_t launch_lincomb(double* out, const double* base, double b, const LinComb& t, long n, hipStream_t s);
// out = (x + y) + z (z may be NULL)
hipError_t launch_combine(const double* x, const double* y, const double* z, double* out, long n, hipStream_t s);

// Batched launches: every workgroup serves the instance block_inst[b].
hipError_t launch_batch_fill_x0(BatchInst* insts, const int* block_inst, int nblocks, hipStream_t s);
hipError_t launch_batch_power_norm(const BatchInst* insts, const int* block_inst, int nblocks, double* partials,
                                   hipStream_t s);
hipError_t launch_batch_power_sweep(const BatchInst* insts, const int* block_inst, int nblocks, double* partials,
                                    int k, hipStream_t s);
hipError_t launch_batch_power_final(BatchInst* insts, int n_inst, const double* partials, int k_last,
                                    double safety, hipStream_t s);
hipError_t launch_batch_coeffs(const BatchInst* insts, int n_inst, const double* xi, double* coef, int ld,
                               hipStream_t s);
// Batched two-iteration launch L (pair.hip; one output per instance, every
// instance with nx even and 16-byte aligned vectors); th in {8, 16};
// burgers: the batch holds a Burgers instance (sizes the LDS for its u tile).
hipError_t launch_batch_pair(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks, bool burgers,
                             int th, double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                             int L, hipStream_t s);
// Batched windows of kBatchBlockDepth iterations (block.hip; one output per
// instance, nx even and sides >= depth, 16-byte aligned vectors, out2 set);
// th 8 or 16 (8 when the batch holds a Burgers instance).
constexpr int kBatchBlockDepth = 4;
hipError_t launch_batch_block(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks, bool burgers,
                              int th, double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                              int L, hipStream_t s);
hipError_t launch_batch_sweep(const BatchInst* insts, LoopCtl* ctls, const int* block_inst, int nblocks,
                              double* partials, const double* coef, int ld, const double* xi, unsigned* done,
                              int m, hipStream_t s);

}  // namespace lx
