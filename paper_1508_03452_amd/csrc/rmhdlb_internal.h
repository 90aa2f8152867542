// rmhdlb_internal.h -- declarations shared by the kernels and the C ABI
// implementation of the HIP library (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmhdlb.h"
#include "rmhdlb_device.h"

namespace rmhd {

constexpr int NPART = 26;  // partial diagnostic sums per block: 9 (see k_moments), 16 Newton bins, fallbacks
constexpr int RED_WAVES = 4;

struct InPtrs {
    const double *n, *p;
    const double *u[3], *E[3], *B[3];
    const double* rho_c;
};

// Prescribed fields of a driven face (nx * ny values each).
struct FacePtrs {
    const double *n, *p;
    const double *u[3], *B[3];
};

struct OutPtrs {
    double *n, *p, *eps;
    double *u[3], *E[3], *B[3], *J[3];
    double* rho_c;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// Deterministic block sums of W values per thread: butterfly within each
// 64-wide wavefront, then the 4 wavefront results in fixed order.  Thread j
// (j < W) writes sum j to out[j].
template <int W>
__device__ __forceinline__ void block_sum(const double (&v)[W], double* __restrict__ out) {
    __shared__ double sh[W][RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const double s = wave_sum(v[j]);
        if (lane == 0) sh[j][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < W) {
        const int j = threadIdx.x;
        out[j] = ((sh[j][0] + sh[j][1]) + (sh[j][2] + sh[j][3]));
    }
}

__device__ __forceinline__ void block_max1(double v, double* __restrict__ out) {
    __shared__ double sh[RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double m = wave_max(v);
    if (lane == 0) sh[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__device__ __forceinline__ double block_sum_value(double v) {
    __shared__ double sh[RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double s = wave_sum(v);
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max_value(double v) {
    __shared__ double sh[RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double m = wave_max(v);
    if (lane == 0) sh[wave] = m;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

int num_tiles(const Consts& K);

// Arrays of the raw (interface) state: F[19], G[19], h*[25], E_prev[3], and
// B_prev[3] with the previous-B reading.
__host__ __device__ inline int state_arrays(const Consts& K) { return NSTATE + (K.bprev ? 3 : 0); }

// Launch shape of the fused step: z-planes walked per block, the tile width
// along x (64, 32 or 16 cells; a row group has 128 cells), the number of
// blocks that walk a column's chunk of zg * zb planes interleaved, and the
// row groups per block stacked along y.
struct StepTuning {
    int zb;
    int px;
    int zg = 1;
    int yw = 1;
};

// One instance of a batched step: its constants, both state buffers (cell
// 0 of the distributions and of E_prev), its face-pass output, its launch
// geometry and its first block and face-pass thread in the batched launches.
struct BatchInst {
    Consts K;
    void* dist[2];
    void* efield[2];
    double* faceB;
    int tiles_x, ncol, zb, yw, nblk;
    int64_t blk0;
    int64_t face0;
};

struct GuessTables;

// Normalisation of the learned guess's inputs and targets (training-set
// mean and standard deviation).
struct Norm4 {
    double mu_x[6], sd_x[6], mu_t[2], sd_t[2];
};

constexpr int SAMPLE_SUMS = 17;  // per-block sums of the sampling pass: F, F^2 (6 each), T, T^2 (2 each), failed

struct TrainArgs {
    const float* X;   // n x 6 normalised inputs
    const float* Yt;  // n x 2 normalised targets
    int n, batch, iters, stride;
    float lr;
    float* w;         // MLP_NP master weights: initial on entry, trained on exit
    float* m;         // Adam moments (zero on entry)
    float* v;
    float* losses;    // loss of every iteration (may be null)
    float* grad;      // gradient-only mode: the gradient of the batch
    float* y;         // gradient-only mode: the outputs, n x 2 (may be null)
    int grad_only;
};



// Device pointers of one state buffer: the 63 distribution arrays and the 3
// E_prev arrays (each `stride` values long).
struct StateBuf {
    void* dist;
    void* efield;
};

// Storage type -> (E_prev storage type, arithmetic type of the step).
template <typename TS>
struct StoreTypes;
template <>
struct StoreTypes<double> {
    using E = double;
    using V = double;
};
template <>
struct StoreTypes<float> {
    using E = float;
    using V = float;
};
template <>
struct StoreTypes<_Float16> {
    using E = float;
    using V = float;
};

// Device buffers of the diagnostics pass.
struct DiagBufs {
    double* faceB;    // adjusted normal B of the open-face cells (Consts::fo layout)
    double* scratch;  // 4 N: B of every cell, then E^z
    double* part;     // NPART per tile
    double* part2;    // max |div B| per tile
    double* nullp;    // (key, cell) per tile
    const double* ez0;  // initial E^z
    const double* b0;   // max |B| of the initial fields
    double* result;   // NPART sums, max |div B|, R, null cell, B0
};

// gt: inference tables of the learned recovery guess, or nullptr for the
// plain recovery (Newton from E_f).
template <typename TS>
hipError_t launch_step(const StateBuf& src, const StateBuf& dst, const Consts& K, const StepTuning& tune,
                       double* faceB, const GuessTables* gt, hipStream_t s);
template <typename TS>
hipError_t launch_moments(const StateBuf& src, const Consts& K, const OutPtrs& out, const DiagBufs& D,
                          const GuessTables* gt, hipStream_t s);
hipError_t launch_init_bmax(const InPtrs& in, const Consts& K, double* part, double* b0, hipStream_t s);
hipError_t launch_face_check(const FacePtrs& in, const Consts& K, double* part, double* result, hipStream_t s);
template <typename TS>
hipError_t launch_ghost(const FacePtrs& in, const Consts& K, const StateBuf& dst, hipStream_t s);
hipError_t launch_init_ref(const InPtrs& in, const Consts& K, double* part, double* result, hipStream_t s);
template <typename TS>
hipError_t launch_face_b(const StateBuf& src, const Consts& K, double* faceB, hipStream_t s);
// Launch geometry of the fused step for a tile width px, zb planes per block
// and zg blocks per column and chunk of zg * zb planes: tiles along x,
// columns, blocks.
void step_geometry(const Consts& K, int px, int zb, int zg, int yw, int cpb, int& tiles_x, int& ncol, int& nblk);
// Cells per row group of a fused-step block: 128 in the pair layout (FP64 storage, two lanes per cell),
// 256 in the quad and double-quad layouts (FP32 and FP16 storage, one lane per cell).
inline int cells_per_block(bool quad) { return quad ? 256 : 128; }
inline bool quad_storage(int32_t storage) { return storage != RMHDLB_STORE_F64; }
// One batched step (face pass of the instances that need it, then the fused
// step of all) reading buffer `parity` of every instance; px the tile width
// (128, 64, 32, 16), waves the occupancy variant (FP32: 2 or 3).
template <typename TS>
hipError_t launch_batch(const BatchInst* dev, int ninst, int total_blocks, int64_t total_face, int px, int waves,
                        int parity, hipStream_t s);
// nsteps batched steps in one cooperative launch of the persistent batch
// kernel (grid barriers between the steps), starting from buffer `parity`;
// next: 16 ints of device memory for its tile counters (cleared here).  No
// face pass: the caller steps batches that need one by graph replays.
template <typename TS>
hipError_t launch_batch_persistent(const BatchInst* dev, int ninst, int total_blocks, int px, int waves, int parity,
                                   int nsteps, int* next, hipStream_t s);
template <typename TS>
hipError_t launch_guess_samples(const StateBuf& src, const Consts& K, double* faceB, int ns, double* F, double* T,
                                double* part, double* result, hipStream_t s);
hipError_t launch_guess_normalise(const double* F, const double* T, int ns, const Norm4& nm, float* X, float* Y,
                                  hipStream_t s);
hipError_t launch_train(const TrainArgs& A, hipStream_t s);
template <typename TS>
hipError_t launch_init(const InPtrs& in, const Consts& K, double* scr, const StateBuf& dst, hipStream_t s);
// Plain copy of n16 16-byte words (the HBM reference rate).
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);
template <typename TS>
hipError_t launch_export(const StateBuf& src, double* dst, const Consts& K, hipStream_t s);
template <typename TS>
hipError_t launch_import(const double* src, const StateBuf& dst, const Consts& K, hipStream_t s);

}  // namespace rmhd
