// rmhdlb_mlp.hip -- training of the learned recovery guess on gfx950:
// sampling of (features, targets) from the solver's own cells, their
// normalisation, and minibatch Adam on a 6 -> 32 -> 32 -> 2 network whose
// forward and backward products run on MFMA (FP16 inputs, FP32 accumulate).
//
// One workgroup of four wavefronts trains (the network has 1346 parameters;
// a wide launch would spend its time in synchronisation): each wavefront
// takes 32 samples at a time, every product is a 32 x 32 tile held in LDS,
// and the gradient is reduced over the four wavefronts in fixed order, so
// training is deterministic.
//
// Tiles are stored row-major as [row][column] in FP16.  Forward and backward
// run transposed (units x samples): Z1^T = W1 X^T, Z2^T = W2 H1^T,
// Y^T = W3 H2^T; dH2^T = W3^T dY^T, dH1^T = W2^T dZ2^T; the weight gradients
// contract over the samples: dW = dZ^T H, db = dZ^T 1.
#include "rmhdlb_device.h"
#include "rmhdlb_internal.h"
#include "rmhdlb_mlp.h"

namespace rmhd {

namespace {

constexpr int TT = 32 * 32;  // elements of a tile
constexpr int TRAIN_WAVES = 4;

// A operand (and B operand of a transposed tile): row = lane % 32, k = 8s + 4h + j.
__device__ __forceinline__ half4 tile_rowk(const _Float16* M, int s) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const half4*>(M + (l & 31) * 32 + 8 * s + 4 * (l >> 5));
}

// B operand of a tile read as [k][n]: column n = lane % 32, k = 8s + 4h + j.
__device__ __forceinline__ half4 tile_colk(const _Float16* M, int s) {
    const int l = threadIdx.x & 63, n = l & 31, k0 = 8 * s + 4 * (l >> 5);
    half4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = M[(k0 + j) * 32 + n];
    return v;
}

// Store a D tile (column lane % 32, item r at row mfma_row(r, lane)).
__device__ __forceinline__ void tile_store(_Float16* M, const floatx16& d) {
    const int l = threadIdx.x & 63, n = l & 31;
#pragma unroll
    for (int r = 0; r < 16; ++r) M[mfma_row(r, l) * 32 + n] = (_Float16)d[r];
}

}  // namespace

__global__ __launch_bounds__(64 * TRAIN_WAVES) void k_train(TrainArgs A) {
    __shared__ __align__(16) _Float16 W1s[TT], W2s[TT], W3s[TT], W2Ts[TT], W3Ts[TT];
    __shared__ float b1s[MLP_H], b2s[MLP_H], b3s[MLP_OUT];
    __shared__ __align__(16) _Float16 work[TRAIN_WAVES][6][TT];  // X, H1, H2, dY, dZ2, dZ1 per wavefront
    __shared__ float lred[TRAIN_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthr = 64 * TRAIN_WAVES;

    // weights into their tiles (zero padding around them)
    for (int i = tid; i < TT; i += nthr) W1s[i] = W2s[i] = W3s[i] = W2Ts[i] = W3Ts[i] = (_Float16)0.0f;
    __syncthreads();
    auto put_param = [&](int t, float val) {
        const _Float16 hv = (_Float16)val;
        if (t < OB1) {
            W1s[(t / MLP_IN) * 32 + t % MLP_IN] = hv;
        } else if (t < OW2) {
            b1s[t - OB1] = val;
        } else if (t < OB2) {
            const int i = (t - OW2) / 32, k = (t - OW2) % 32;
            W2s[i * 32 + k] = hv;
            W2Ts[k * 32 + i] = hv;
        } else if (t < OW3) {
            b2s[t - OB2] = val;
        } else if (t < OB3) {
            const int o = (t - OW3) / 32, k = (t - OW3) % 32;
            W3s[o * 32 + k] = hv;
            W3Ts[k * 32 + o] = hv;
        } else {
            b3s[t - OB3] = val;
        }
    };
    for (int t = tid; t < MLP_NP; t += nthr) put_param(t, A.w[t]);

    half4 ones;
#pragma unroll
    for (int j = 0; j < 4; ++j) ones[j] = (_Float16)1.0f;
    const int nchunk = A.batch / 32;  // a multiple of TRAIN_WAVES (the host checks)
    const int iters = A.grad_only ? 1 : A.iters;
    const float inv_batch = 1.0f / (float)A.batch;
    _Float16* MX = work[wave][0];
    _Float16* MH1 = work[wave][1];
    _Float16* MH2 = work[wave][2];
    _Float16* MdY = work[wave][3];
    _Float16* MdZ2 = work[wave][4];
    _Float16* MdZ1 = work[wave][5];
    const int c = lane & 31, hh = lane >> 5;

    for (int it = 0; it < iters; ++it) {
        for (int i = tid; i < TRAIN_WAVES * 6 * TT; i += nthr) (&work[0][0][0])[i] = (_Float16)0.0f;
        __syncthreads();
        floatx16 gW1 = {0}, gb1 = {0}, gW2 = {0}, gb2 = {0}, gW3 = {0}, gb3 = {0};
        float lacc = 0.0f;
        for (int q = wave; q < nchunk; q += TRAIN_WAVES) {
            const int slot = q * 32 + c;
            const int idx = A.grad_only ? slot : (int)(((int64_t)it * A.batch + slot) * A.stride % A.n);
#pragma unroll
            for (int j = 0; j < 3; ++j) MX[(3 * hh + j) * 32 + c] = (_Float16)A.X[(int64_t)idx * MLP_IN + 3 * hh + j];
            __syncthreads();
            // forward
            floatx16 d = {0};
            d = mfma_32x32x8(tile_rowk(W1s, 0), tile_colk(MX, 0), d);
            floatx16 H1;
#pragma unroll
            for (int r = 0; r < 16; ++r) H1[r] = fast_tanh(d[r] + b1s[mfma_row(r, lane)]);
            tile_store(MH1, H1);
            __syncthreads();
            floatx16 e = {0};
#pragma unroll
            for (int s = 0; s < 4; ++s) e = mfma_32x32x8(tile_rowk(W2s, s), tile_colk(MH1, s), e);
            floatx16 H2;
#pragma unroll
            for (int r = 0; r < 16; ++r) H2[r] = fast_tanh(e[r] + b2s[mfma_row(r, lane)]);
            tile_store(MH2, H2);
            __syncthreads();
            floatx16 o = {0};
#pragma unroll
            for (int s = 0; s < 4; ++s) o = mfma_32x32x8(tile_rowk(W3s, s), tile_colk(MH2, s), o);
            // loss and dL/dY (rows 0, 1 of column c are items 0, 1 of lane c)
            floatx16 dY = {0};
            if (lane < 32) {
#pragma unroll
                for (int k = 0; k < MLP_OUT; ++k) {
                    const float y = o[k] + b3s[k];
                    const float r = y - A.Yt[(int64_t)idx * MLP_OUT + k];
                    lacc += r * r;
                    dY[k] = r * inv_batch;
                    if (A.grad_only && A.y) A.y[(int64_t)idx * MLP_OUT + k] = y;
                }
            }
            tile_store(MdY, dY);
            __syncthreads();
            // backward
            floatx16 g2 = {0};
            g2 = mfma_32x32x8(tile_rowk(W3Ts, 0), tile_colk(MdY, 0), g2);  // outputs 0..7 cover the 2 real ones
            floatx16 dZ2;
#pragma unroll
            for (int r = 0; r < 16; ++r) dZ2[r] = g2[r] * (1.0f - H2[r] * H2[r]);
            tile_store(MdZ2, dZ2);
            __syncthreads();
            floatx16 g1 = {0};
#pragma unroll
            for (int s = 0; s < 4; ++s) g1 = mfma_32x32x8(tile_rowk(W2Ts, s), tile_colk(MdZ2, s), g1);
            floatx16 dZ1;
#pragma unroll
            for (int r = 0; r < 16; ++r) dZ1[r] = g1[r] * (1.0f - H1[r] * H1[r]);
            tile_store(MdZ1, dZ1);
            __syncthreads();
            // weight and bias gradients: contractions over the 32 samples
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const half4 ay = tile_rowk(MdY, s), a2 = tile_rowk(MdZ2, s), a1 = tile_rowk(MdZ1, s);
                gW3 = mfma_32x32x8(ay, tile_rowk(MH2, s), gW3);
                gb3 = mfma_32x32x8(ay, ones, gb3);
                gW2 = mfma_32x32x8(a2, tile_rowk(MH1, s), gW2);
                gb2 = mfma_32x32x8(a2, ones, gb2);
                gW1 = mfma_32x32x8(a1, tile_rowk(MX, s), gW1);
                gb1 = mfma_32x32x8(a1, ones, gb1);
            }
            __syncthreads();
        }
        // per-wavefront gradients into LDS (the work tiles are free now), then
        // the sum over wavefronts in fixed order
        float* G = reinterpret_cast<float*>(&work[0][0][0]);
        float* Gw = G + wave * MLP_NP;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = mfma_row(r, lane);
            if (c < MLP_IN) Gw[OW1 + i * MLP_IN + c] = gW1[r];
            Gw[OW2 + i * 32 + c] = gW2[r];
            if (i < MLP_OUT) Gw[OW3 + i * 32 + c] = gW3[r];
            if (c == 0) {
                Gw[OB1 + i] = gb1[r];
                Gw[OB2 + i] = gb2[r];
                if (i < MLP_OUT) Gw[OB3 + i] = gb3[r];
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) lacc += __shfl_xor(lacc, off, 64);
        if (lane == 0) lred[wave] = lacc;
        __syncthreads();
        const float b1p = 1.0f - powf(0.9f, (float)(it + 1)), b2p = 1.0f - powf(0.999f, (float)(it + 1));
        for (int t = tid; t < MLP_NP; t += nthr) {
            const float g = ((G[t] + G[MLP_NP + t]) + G[2 * MLP_NP + t]) + G[3 * MLP_NP + t];
            if (A.grad_only) {
                A.grad[t] = g;
            } else {
                const float m = 0.9f * A.m[t] + 0.1f * g;
                const float v = 0.999f * A.v[t] + 0.001f * g * g;
                A.m[t] = m;
                A.v[t] = v;
                const float w = A.w[t] - A.lr * (m / b1p) / (sqrtf(v / b2p) + 1e-8f);
                A.w[t] = w;
                put_param(t, w);
            }
        }
        if (tid == 0 && A.losses) A.losses[it] = 0.5f * ((lred[0] + lred[1]) + (lred[2] + lred[3])) * inv_batch;
        __syncthreads();
    }
}

__global__ void k_guess_normalise(const double* __restrict__ F, const double* __restrict__ T, int ns, Norm4 nm,
                                  float* __restrict__ X, float* __restrict__ Y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ns) return;
#pragma unroll
    for (int j = 0; j < 6; ++j) X[(int64_t)i * 6 + j] = (float)((F[(int64_t)i * 6 + j] - nm.mu_x[j]) / nm.sd_x[j]);
#pragma unroll
    for (int k = 0; k < 2; ++k) Y[(int64_t)i * 2 + k] = (float)((T[(int64_t)i * 2 + k] - nm.mu_t[k]) / nm.sd_t[k]);
}

hipError_t launch_guess_normalise(const double* F, const double* T, int ns, const Norm4& nm, float* X, float* Y,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_guess_normalise, dim3((ns + 255) / 256), dim3(256), 0, s, F, T, ns, nm, X, Y);
    return hipGetLastError();
}

hipError_t launch_train(const TrainArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_train, dim3(1), dim3(64 * TRAIN_WAVES), 0, s, A);
    return hipGetLastError();
}

}  // namespace rmhd
