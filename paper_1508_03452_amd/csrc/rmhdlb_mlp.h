// rmhdlb_mlp.h -- the learned recovery guess on gfx950: a 6 -> 32 -> 32 -> 2
// perceptron (tanh hidden layers, linear output) evaluated with FP16-input,
// FP32-accumulate MFMA (v_mfma_f32_32x32x16_f16 in the step's inference,
// v_mfma_f32_32x32x8_f16 in training), 32 cells per wavefront.
//
// The network seeds the Newton iteration of the Landau-frame recovery with a
// guess of the eigenvalue; Newton still converges to the same root, so the
// guess changes the iteration count, never the result.  (Not in the paper,
// whose recovery is the power method, Sec. III coupling subsection.)
//
// Inputs (rotation and scale invariants of the fluid tensor, E_f = T_fl^00,
// S = T_fl^0a, Pi = T_fl^ab, S_hat = S / |S| or 0):
//   |S|/E_f, S_hat.Pi.S_hat/E_f, tr Pi/E_f, |Pi S_hat - (S_hat.Pi.S_hat) S_hat|/E_f,
//   |Pi|_F/E_f, N^0/E_f, then normalised with training-set mean and deviation.
// Outputs (normalised): lambda / E_f and |beta|.
//
// Layout conventions of v_mfma_f32_32x32x8_f16 on a 64-wide wavefront, lane l,
// h = l / 32: A (32 x 8) row l % 32, k = 4 h + j; B (8 x 32) column l % 32,
// k = 4 h + j (j = 0..3, one half4 each); D (32 x 32) column l % 32, item r
// holds row 8 (r / 4) + 4 h + r % 4.  v_mfma_f32_32x32x16_f16 takes K = 16:
// A row l % 32, k = 8 h + j, B column l % 32, k = 8 h + j (j = 0..7, one
// half8 each), D as above.  Layers are evaluated transposed (units x cells,
// D = W X^T).  A contraction may take its K index in any order that A and B
// share, so K-step s of the next layer contracts over the rows that a lane's
// D items 8s..8s+7 hold (rows 8 (2s + j / 4) + 4 h + j % 4), the weights are
// packed in that order, and the activations never leave the registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmhd {

constexpr int MLP_IN = 6, MLP_H = 32, MLP_OUT = 2;
constexpr int MLP_NP = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 1346
// offsets in the flat parameter vector W1 (32 x 6), b1, W2 (32 x 32), b2, W3 (2 x 32), b3
constexpr int OW1 = 0, OB1 = OW1 + MLP_H * MLP_IN, OW2 = OB1 + MLP_H, OB2 = OW2 + MLP_H * MLP_H, OW3 = OB2 + MLP_H,
              OB3 = OW3 + MLP_OUT * MLP_H;

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Per-lane operand tables of the inference (built on the host from the weights).
struct GuessTables {
    half8 a1[64];     // layer-1 A operand (W1 padded to 32 x 16)
    half8 a2[64][2];  // layer-2 A operands, K-steps 0..1 (k in the order of guess_k)
    half8 a3[64][2];  // layer-3 A operands (W3 padded to 32 rows)
    float b1[64][16]; // bias of D item r of each lane
    float b2[64][16];
    float b3[2];
    float mu_x[6], inv_sd_x[6];
    float mu_t[2], sd_t[2];
};

// Row of item r of a D tile held by lane l.
__host__ __device__ constexpr int mfma_row(int r, int lane) { return 8 * (r / 4) + 4 * ((lane >> 5) & 1) + (r & 3); }
// Unit contracted at position j of K-step s of a hidden or output layer in lane l (the row of the
// previous layer's D item 8s + j).
__host__ __device__ constexpr int guess_k(int s, int j, int lane) { return mfma_row(8 * s + j, lane); }

// |S| and the first invariant |S| / E_f, the flow measure the guess is gated on.
__device__ __forceinline__ double flow_ratio(double Ef, const double S[3], double& s) {
    s = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    return s * (1.0 / Ef);
}

// The six invariants of a fluid tensor (FP64; Pi as xx, yy, zz, xy, xz, yz), given |S| and f[0]
// from flow_ratio.
__device__ __forceinline__ void mlp_features(double Ef, const double S[3], const double Pi[6], double N0,
                                             double s, double f[6]) {
    const double is = s > 0.0 ? 1.0 / s : 0.0;
    const double h0 = S[0] * is, h1 = S[1] * is, h2 = S[2] * is;
    const double p0 = Pi[0] * h0 + Pi[3] * h1 + Pi[4] * h2;
    const double p1 = Pi[3] * h0 + Pi[1] * h1 + Pi[5] * h2;
    const double p2 = Pi[4] * h0 + Pi[5] * h1 + Pi[2] * h2;
    const double sps = h0 * p0 + h1 * p1 + h2 * p2;
    const double q0 = p0 - sps * h0, q1 = p1 - sps * h1, q2 = p2 - sps * h2;
    const double fro = sqrt(Pi[0] * Pi[0] + Pi[1] * Pi[1] + Pi[2] * Pi[2] +
                            2.0 * (Pi[3] * Pi[3] + Pi[4] * Pi[4] + Pi[5] * Pi[5]));
    const double ie = 1.0 / Ef;
    f[1] = sps * ie;
    f[2] = (Pi[0] + Pi[1] + Pi[2]) * ie;
    f[3] = sqrt(q0 * q0 + q1 * q1 + q2 * q2) * ie;
    f[4] = fro * ie;
    f[5] = N0 * ie;
}

// tanh through the hardware exponential: 1 - 2 / (1 + e^{2x}) (saturates to +-1).
__device__ __forceinline__ float fast_tanh(float x) { return 1.0f - 2.0f / (1.0f + __expf(2.0f * x)); }

__device__ __forceinline__ floatx16 mfma_32x32x8(half4 a, half4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x8f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx16 mfma_32x32x16(half8 a, half8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ half4 to_half4(float a, float b, float c, float d) {
    half4 v;
    v[0] = (_Float16)a;
    v[1] = (_Float16)b;
    v[2] = (_Float16)c;
    v[3] = (_Float16)d;
    return v;
}

// tanh of (D item + bias) for the 8 items 8s..8s+7 of a tile, as the next layer's B operand.
__device__ __forceinline__ half8 act8(const floatx16& d, const float* __restrict__ bias, int s) {
    half8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (_Float16)fast_tanh(d[8 * s + j] + bias[8 * s + j]);
    return v;
}

// Network outputs (normalised) for 32 cells of a wavefront.  Every lane of
// the wavefront must call this together.  x[6] are the normalised inputs of
// this lane's own cell; column n of the product takes them from lane
// src_lane(n); the outputs of this lane's cell are read from lane out_lane.
__device__ __forceinline__ void mlp_wave(const GuessTables* __restrict__ T, const float x[6], int src_lane,
                                         int out_lane, float& y0, float& y1) {
    const int lane = threadIdx.x & 63, h = lane >> 5;
    float g[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) g[j] = __shfl(x[j], src_lane, 64);
    half8 b0 = {0};
    if (h == 0) {
#pragma unroll
        for (int j = 0; j < 6; ++j) b0[j] = (_Float16)g[j];
    }
    floatx16 d = {0};
    d = mfma_32x32x16(T->a1[lane], b0, d);
    const half8 h0 = act8(d, T->b1[lane], 0), h1 = act8(d, T->b1[lane], 1);
    floatx16 e = {0};
    e = mfma_32x32x16(T->a2[lane][0], h0, e);
    e = mfma_32x32x16(T->a2[lane][1], h1, e);
    const half8 k0 = act8(e, T->b2[lane], 0), k1 = act8(e, T->b2[lane], 1);
    floatx16 o = {0};
    o = mfma_32x32x16(T->a3[lane][0], k0, o);
    o = mfma_32x32x16(T->a3[lane][1], k1, o);
    // rows 0 and 1 of column n are items 0 and 1 of lane n (n < 32)
    y0 = __shfl(o[0] + T->b3[0], out_lane, 64);
    y1 = __shfl(o[1] + T->b3[1], out_lane, 64);
}

}  // namespace rmhd
