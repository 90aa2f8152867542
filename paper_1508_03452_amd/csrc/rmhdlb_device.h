// rmhdlb_device.h -- device-side lattice tables and per-cell physics of the
// resistive relativistic MHD lattice Boltzmann step (arXiv:1508.03452,
// Sec. III), written for gfx950 in FP64 arithmetic.
//
// The fluid distributions are held in the normalised, nu-free variables
// F = (c_t/c_0)^2 f and G = (c_t/c_0) g, for which the moments are
// T^00 = sum F, T^0a = kappa sum e^a F, T^ab = kappa^2 sum e^a e^b F and
// N^0 = sum G, with kappa = c_0 c_a / c_t = sqrt(19/27).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmhd {

// ---------------------------------------------------------------- lattices

constexpr int Q = 19;   // D3Q19 (Eq. cellconfigs1)
constexpr int QH = 24;  // moving D3Q13 Maxwell populations; index 24 is the rest one
constexpr int NSTATE = Q + Q + QH + 1 + 3;  // F, G, h*, E_prev

// Interface order of the D3Q19 directions: rest, +-x, +-y, +-z, then the
// face diagonals in the xy, xz and yz planes.
constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// D3Q19 weights: they do not depend on nu (Sec. III): -44/361, 99/722, 9/361.
__host__ __device__ constexpr double weight(int i) {
    return i == 0 ? -44.0 / 361.0 : (i <= 6 ? 99.0 / 722.0 : 9.0 / 361.0);
}

// D3Q13 Maxwell lattice, population k = 8 p + 2 i + j (plane p = xy, xz, yz;
// direction i; auxiliary pair j).  v_k dt = (SX, SY, SZ) dx, i.e. v_k =
// sqrt(2) c s_k; e_k = (c / sqrt 2) ehat_k; b_k = bhat_k.  The pair j = 1 has
// the opposite e and b of j = 0.
constexpr int SX[QH] = {1, 1, -1, -1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0};
constexpr int SY[QH] = {1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1};
constexpr int SZ[QH] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int EHX[QH] = {1, -1, 1, -1, -1, 1, -1, 1, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0};
constexpr int EHY[QH] = {-1, 1, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1};
constexpr int EHZ[QH] = {0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 1, -1, -1, 1, -1, 1, 1, -1, 1, -1, -1, 1};
constexpr int BHX[QH] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1};
constexpr int BHY[QH] = {0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 0, 0, 0, 0};
constexpr int BHZ[QH] = {-1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

// Offsets of the state arrays (each `stride` values long); E_prev (OFF_E..)
// lives in its own block of the buffer.
constexpr int OFF_F = 0, OFF_G = Q, OFF_H = 2 * Q, OFF_E = 2 * Q + QH + 1;

// --------------------------------------------------------------- constants

struct Consts {
    int nx, ny, nz;
    int per[3];          // 1 = periodic axis, 0 = open or driven
    int drv;             // 1: driven low z face, ghost planes z = -1, -2 stored below the interior
    int divb;            // 1: the normal B of open-face cells is adjusted so that div B = 0 there
    int open_lo[3], open_hi[3];  // face takes the div B adjustment (open, with at least 2 cells on the axis)
    int band;            // half-width in rows of the reconnection null search band
    int64_t fo[7];       // offsets of the six face arrays of adjusted normal B (x lo, x hi, y lo, ...), fo[6] = total
    int64_t N;           // cells
    int64_t stride;      // values per state array (ghost planes + N, rounded up)
    int64_t g0;          // ghost cells in front of cell 0 of every array
    double c, dx, eps0;
    double cour;         // Courant number along a link: kappa c dt / dx
    double kv;           // bulk-viscosity coefficient alpha c dt / dx
    double inv_tau;      // 1 / tau (tau in units of dt)
    double wg;           // rate of the g collision, (c_0 nu / c_t) / tau
    double q;            // (dt / 2) mu0 c^2
    double sigma, gm1;   // conductivity, Gamma - 1
    double wp[3];        // g weights (rest, axis, diagonal)
    double gc1, gc2, gc3;  // (c_t/c_0) * (3 c_a, 9/2 c_a^2, 3/2) of the g equilibrium
    double inv_2dx;
    // Stored f, g are deviations from these per-class shifts (rest, axis,
    // diagonal): w_i E_ref and w'_i N_ref rounded to the step's arithmetic
    // type, all 0 on the plain FP64 path.  fs0 = sum_i fsh_i, fsaa = the sum
    // over the directions with e^a != 0 (any axis a), gs0 = sum_i gsh_i.
    double fsh[3], gsh[3];
    double fs0, fsaa, gs0;
    // the alternative readings (the host picks the kernel variant from coll, flux)
    double slope;        // weight of the limited slope in a face value: 1/2 (MUSCL) or (1 - cour)/2 (Lax-Wendroff)
    int coll;            // f collision: 0 explicit, 1 the printed semi-implicit form
    int flux;            // face values: 0 MUSCL, 1 limited Lax-Wendroff
    int bprev;           // 1: the previous step's B in the recovery and f_eq; the field block then holds
                         // E_prev[3] and B_prev[3] (else E_prev[3] only)
    // external force density (3 arrays of N, cell order) and its gate: on while
    // the previous step's largest |beta| (*vmax_prev) is below fgate (<= 0: always)
    int forced;
    double fgate;
    const double* force;
    const double* vmax_prev;
    double* vmax_part;   // largest |beta| per wavefront of the step, reduced after it
    // gate of the learned guess (set per launch): a step runs the network only
    // when the step before it met a cell whose flow ratio |S| / E_f exceeds the
    // gate, i.e. when *gflag_rd == gstep - 1; a step that meets one stores its
    // number gstep in *gflag_wr (null: record nothing).  Two slots, swapped
    // with the state buffers.
    const int64_t* gflag_rd;
    int64_t* gflag_wr;
    int64_t gstep;
    int64_t* gcount;     // steps that ran the network (null: not counted)
};

// Layout of the distributions in a state buffer.  Element indices are
// relative to the buffer's distribution pointer, which sits g0 elements into
// the buffer (the ghost planes of a driven face take the g0 positions in
// front of cell 0 of every array; position p = g0 + c of cell c).
//  - FP64 (pair layout): direction i as pairs (f_i, g_i), pair of cell c at
//    2 (i S + p); Maxwell population k as its own array at (38 + k) S + p.
//  - FP32 (quad layout): direction slot s = 1..9 holds the opposite
//    directions 2s - 1 (e) and 2s (-e) as quads (f_{2s-1}, g_{2s-1}, f_{2s},
//    g_{2s}) at 4 (s S + p), slot 0 the rest pair (f_0, g_0, 0, 0); the moving
//    Maxwell populations 2m and 2m + 1, which stream from the same cell, as
//    pairs at 40 S + 2 (m S + p), the rest one at 64 S + p.  One lane then
//    reads both directions of a slot, and both populations of a pair, with one
//    load per stencil point.
//  - FP16 (double-quad layout): the quads of two slots side by side in one
//    16-byte record, record r = 0..3 holding slots 2r + 1 and 2r + 2, record
//    4 slot 9 and the rest pair (f_0, g_0, 0, 0), at 8 (r S + p); the Maxwell
//    populations as in the quad layout.  The centre point and the six
//    Laplacian points of two slots then take one load.
constexpr int QUAD_SLOTS = 10;           // quad layout: 40 S elements of f and g
constexpr int QUAD_DIST_ARRAYS = 65;     // quad layout: distribution block of 65 S elements
constexpr int PAIR_DIST_ARRAYS = 63;     // pair layout: 38 S of f, g and 25 S of h
__host__ __device__ inline int64_t quad_index(const Consts& K, int slot, int64_t c) {
    return 4 * ((int64_t)slot * K.stride + c) + 3 * K.g0;
}
__host__ __device__ inline int64_t hpair_index(const Consts& K, int m, int64_t c) {
    return 4 * (int64_t)QUAD_SLOTS * K.stride + 2 * ((int64_t)m * K.stride + c) + K.g0;
}
__host__ __device__ inline int64_t hrest_quad_index(const Consts& K, int64_t c) {
    return (4 * (int64_t)QUAD_SLOTS + QH) * K.stride + c;
}
// Direction i of the quad layout: its slot and its position (0 or 2) in the quad.
__host__ __device__ constexpr int quad_slot(int i) { return (i + 1) / 2; }
__host__ __device__ constexpr int quad_pos(int i) { return (i == 0 || (i & 1)) ? 0 : 2; }
// Double-quad layout: record r of cell c, and slot s's record and offset (0 or 4) in it.
constexpr int DQUAD_RECORDS = 5;
__host__ __device__ inline int64_t dquad_index(const Consts& K, int r, int64_t c) {
    return 8 * ((int64_t)r * K.stride + c) + 7 * K.g0;
}
__host__ __device__ constexpr int dquad_rec(int s) { return s == 0 ? 4 : (s - 1) / 2; }
__host__ __device__ constexpr int dquad_off(int s) { return s == 0 ? 4 : (s == 9 ? 0 : ((s - 1) & 1) * 4); }
static_assert(8 * DQUAD_RECORDS == 4 * QUAD_SLOTS, "the Maxwell block follows the same 40 S elements");

// The pairings the quad layout relies on: slot s holds e_{2s-1} and its opposite; the Maxwell
// populations 2m and 2m + 1 share the streaming offset and have opposite e and b.
__host__ __device__ constexpr bool quad_pairings_hold() {
    for (int s = 1; s <= 9; ++s)
        if (EX[2 * s] != -EX[2 * s - 1] || EY[2 * s] != -EY[2 * s - 1] || EZ[2 * s] != -EZ[2 * s - 1]) return false;
    for (int m = 0; m < 12; ++m) {
        const int a = 2 * m, b = 2 * m + 1;
        if (SX[a] != SX[b] || SY[a] != SY[b] || SZ[a] != SZ[b]) return false;
        if (EHX[a] != -EHX[b] || EHY[a] != -EHY[b] || EHZ[a] != -EHZ[b]) return false;
        if (BHX[a] != -BHX[b] || BHY[a] != -BHY[b] || BHZ[a] != -BHZ[b]) return false;
    }
    return true;
}
static_assert(quad_pairings_hold(), "the lattice tables no longer pair opposite directions");

constexpr double KAPPA = 0.83887049280786108;   // sqrt(19/27)
constexpr double KAPPA2 = 19.0 / 27.0;
constexpr double SQRT19_3 = 2.5166114784235836; // sqrt(19/3)
constexpr double INV_SQRT2 = 0.70710678118654752;

// ------------------------------------------------------------- primitives

template <typename V>
__device__ __forceinline__ V minmod(V a, V b) {
    if (a * b <= V(0)) return V(0);
    return fabs(a) < fabs(b) ? a : b;
}

// Solve (Pi + lam I) y = S for the symmetric 3x3 Pi (xx, yy, zz, xy, xz, yz)
// by cofactors.
__device__ __forceinline__ void solve_shifted(const double Pi[6], double lam, const double S[3], double y[3]) {
    const double a = Pi[0] + lam, b = Pi[1] + lam, c = Pi[2] + lam;
    const double d = Pi[3], e = Pi[4], f = Pi[5];
    const double c00 = b * c - f * f, c01 = e * f - d * c, c02 = d * f - e * b;
    const double c11 = a * c - e * e, c12 = d * e - a * f, c22 = a * b - d * d;
    const double inv = 1.0 / (a * c00 + d * c01 + e * c02);
    y[0] = (c00 * S[0] + c01 * S[1] + c02 * S[2]) * inv;
    y[1] = (c01 * S[0] + c11 * S[1] + c12 * S[2]) * inv;
    y[2] = (c02 * S[0] + c12 * S[1] + c22 * S[2]) * inv;
}

// (Pi + lam I) y = S with a positive-definiteness test of Pi + lam I (its
// leading principal minors).
__device__ __forceinline__ bool solve_shifted_pd(const double Pi[6], double lam, const double S[3], double y[3]) {
    const double a = Pi[0] + lam, b = Pi[1] + lam, c = Pi[2] + lam;
    const double d = Pi[3], e = Pi[4], f = Pi[5];
    const double c00 = b * c - f * f, c01 = e * f - d * c, c02 = d * f - e * b;
    const double c11 = a * c - e * e, c12 = d * e - a * f, c22 = a * b - d * d;
    const double det = a * c00 + d * c01 + e * c02;
    const double inv = 1.0 / det;
    y[0] = (c00 * S[0] + c01 * S[1] + c02 * S[2]) * inv;
    y[1] = (c01 * S[0] + c11 * S[1] + c12 * S[2]) * inv;
    y[2] = (c02 * S[0] + c12 * S[1] + c22 * S[2]) * inv;
    return a > 0.0 && c22 > 0.0 && det > 0.0;
}

// Landau-frame recovery.  The fluid tensor T_fl = T - T_EM has the timelike
// eigenvector (1, beta) with eigenvalue eps: (Pi + eps I) beta = S and
// eps = E_f - S.beta.  Eliminating beta gives the secular equation
// phi(lam) = lam - E_f + S^T (Pi + lam I)^-1 S = 0, convex where Pi + lam I
// is positive definite and increasing above its minimum (phi' = 1 - |beta|^2
// = 1/gamma^2 at the root).  Newton from a start on the increasing branch
// passes the root at most once (from below) and then decreases
// monotonically to it.  Every Newton step is applied (so lam carries no
// one-sided bias) until the step is at the rounding floor; beta is then
// solved at the final lam.  Returns the number of Newton steps.  With SOLVED,
// beta already holds the solution at lam0 (the first solve is skipped).
template <bool SOLVED = false>
__device__ __forceinline__ int newton_from(double Ef, const double S[3], const double Pi[6], double lam0,
                                           double& lam, double beta[3]) {
    lam = lam0;
    int it = 0;
    while (it < 60) {
        if (!SOLVED || it > 0) solve_shifted(Pi, lam, S, beta);
        const double phi = lam - Ef + (S[0] * beta[0] + S[1] * beta[1] + S[2] * beta[2]);
        const double dphi = 1.0 - (beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2]);
        const double d = phi / dphi;
        ++it;
        if (d == 0.0) return it;  // beta already solved at lam
        lam -= d;
        if (!(fabs(d) > 4.5e-16 * fabs(lam))) break;
    }
    solve_shifted(Pi, lam, S, beta);
    return it;
}

// Plain start: lam = E_f, where phi = S^T (Pi + E_f I)^-1 S >= 0.
__device__ __forceinline__ int recover(double Ef, const double S[3], const double Pi[6], double& lam,
                                       double beta[3]) {
    return newton_from(Ef, S, Pi, Ef, lam, beta);
}

// Start from a guess lam0 when it lies below E_f on the increasing branch of
// phi (Pi + lam0 I positive definite, phi'(lam0) > 0); otherwise from E_f,
// with fallback = 1 (lam0 = E_f means no guess was offered: fallback = 0).
__device__ __forceinline__ int recover_from_guess(double Ef, const double S[3], const double Pi[6], double lam0,
                                                  double& lam, double beta[3], int& fallback) {
    fallback = lam0 == Ef ? 0 : 1;
    if (lam0 < Ef) {  // false for NaN
        const bool pd = solve_shifted_pd(Pi, lam0, S, beta);  // the same solve as Newton's first one
        if (pd && 1.0 - (beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2]) > 0.0) {
            fallback = 0;
            return newton_from<true>(Ef, S, Pi, lam0, lam, beta);
        }
    }
    return recover(Ef, S, Pi, lam, beta);
}

}  // namespace rmhd
