// rmhdlb_kernels.hip -- gfx950 kernels of the resistive relativistic MHD
// lattice Boltzmann step (arXiv:1508.03452, Sec. III).
//
// Layout in HBM: structure of arrays, x fastest.  A state buffer holds the
// distributions F[0..18], G[0..18], h*[0..24] of storage type TS, interleaved
// as (f_i, g_i) pairs (FP64, 63 arrays), as quads of opposite directions
// (FP32, 65 arrays) or as records of two such quads (FP16, 65 arrays; the
// layouts are described in rmhdlb_device.h),
// then (256-byte aligned) the 3 E_prev arrays of type TE (TS, or FP32 when TS
// is FP16); two buffers, read one and write the other.  The stored state is post-collision.  On the FP32 and FP16
// storage paths F and G are stored as deviations from w_i E_ref and
// w'_i N_ref (references from the initial fields) and the step runs in FP32
// arithmetic, with the recovery and the Ohm solve in FP64.
#include <hip/hip_cooperative_groups.h>

#include "rmhdlb_device.h"
#include "rmhdlb_internal.h"
#include "rmhdlb_mlp.h"

namespace rmhd {

constexpr int TX = 64, TY = 4, TPB = TX * TY;

template <typename T>
__device__ __forceinline__ double ld(const T* __restrict__ p, int64_t i) {
    return static_cast<double>(p[i]);
}

template <typename V, typename T>
__device__ __forceinline__ V ldv(const T* __restrict__ p, int64_t i) {
    return static_cast<V>(p[i]);
}

// Loads of values that no other cell of the step reads (each streamed h* is
// pulled by exactly one cell): the non-temporal hint keeps them from
// evicting the stencil lines that the neighbours' loads will hit.  Used for
// 4- and 8-byte values only: a 2-byte array shares each cache line between
// two wavefronts, and the hint then costs the second one a refetch.
template <typename V, typename T>
__device__ __forceinline__ V ldv_once(const T* __restrict__ p, int64_t i) {
    if constexpr (sizeof(T) >= 4)
        return static_cast<V>(__builtin_nontemporal_load(p + i));
    else
        return static_cast<V>(p[i]);
}

// Stores of the next state are never read again in this step: the
// non-temporal hint keeps them from evicting the stencil lines from L2.
template <bool NT, typename T, typename V>
__device__ __forceinline__ void st(T* __restrict__ p, V v) {
    if constexpr (NT)
        __builtin_nontemporal_store(static_cast<T>(v), p);
    else
        *p = static_cast<T>(v);
}

// f and g of one direction are stored interleaved: the pair (f_i, g_i) of
// cell c sits at fg[2 (i S + c)], fg = dist + g0 (the f-g block spans the
// first 38 S values; ghost cells in front of cell 0 take 2 g0 of them).
// Both use the same transport stencil, so one vector load serves both.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t fg_index(const Consts& K, int i, int64_t c) {
    return 2 * ((int64_t)i * K.stride + c) + K.g0;
}

template <typename V, typename T>
__device__ __forceinline__ vec2<V> ldv2(const T* __restrict__ p, int64_t i) {
    const vec2<T> v = *reinterpret_cast<const vec2<T>*>(p + i);
    vec2<V> r;
    r.x = static_cast<V>(v.x);
    r.y = static_cast<V>(v.y);
    return r;
}

template <bool NT, typename T, typename V>
__device__ __forceinline__ void st2(T* __restrict__ p, V f, V g) {
    vec2<T> v;
    v.x = static_cast<T>(f);
    v.y = static_cast<T>(g);
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<vec2<T>*>(p));
    else
        *reinterpret_cast<vec2<T>*>(p) = v;
}

// FP64 storage uses the pair layout (two lanes per cell), FP32 the quad and
// FP16 the double-quad layout (one lane per cell; see rmhdlb_device.h).
// Element indices of f_i, g_i and h_k of cell c (c may be a ghost cell of a
// driven face, down to -g0), for the kernels that read or write single values.
template <typename TS>
constexpr bool quad_layout() {  // one lane per cell
    return sizeof(TS) != 8;
}
template <typename TS>
constexpr bool dquad_layout() {
    return sizeof(TS) == 2;
}
// Element index of the quad of slot s of cell c in the quad and double-quad layouts.
template <typename TS>
__host__ __device__ __forceinline__ int64_t slot_index(const Consts& K, int s, int64_t c) {
    if constexpr (dquad_layout<TS>())
        return dquad_index(K, dquad_rec(s), c) + dquad_off(s);
    else
        return quad_index(K, s, c);
}
template <typename TS>
__device__ __forceinline__ int64_t f_at(const Consts& K, int i, int64_t c) {
    if constexpr (quad_layout<TS>())
        return slot_index<TS>(K, quad_slot(i), c) + quad_pos(i);
    else
        return fg_index(K, i, c);
}
template <typename TS>
__device__ __forceinline__ int64_t g_at(const Consts& K, int i, int64_t c) {
    return f_at<TS>(K, i, c) + 1;
}
template <typename TS>
__device__ __forceinline__ int64_t h_at(const Consts& K, int k, int64_t c) {
    if constexpr (quad_layout<TS>())
        return k < QH ? hpair_index(K, k / 2, c) + (k & 1) : hrest_quad_index(K, c);
    else
        return (int64_t)(OFF_H + k) * K.stride + c;
}

// Shift of the stored f, g of direction i (0 on the plain FP64 path).
__device__ __forceinline__ double fshift(const Consts& K, int i) { return K.fsh[i == 0 ? 0 : (i <= 6 ? 1 : 2)]; }
__device__ __forceinline__ double gshift(const Consts& K, int i) { return K.gsh[i == 0 ? 0 : (i <= 6 ? 1 : 2)]; }

// Neighbour offsets of one cell along one axis for displacements -2..+2,
// with periodic wrap or (open face) a copy of the first interior cell; with
// keep_low the coordinates -1, -2 stay (the ghost planes of a driven face).
__device__ __forceinline__ int map_coord(int v, int n, int periodic, int keep_low) {
    if (v < 0) return periodic ? (v + n >= 0 ? v + n : v + 2 * n) : (keep_low ? v : 0);
    if (v >= n) return periodic ? (v - n < n ? v - n : v - 2 * n) : n - 1;
    return v;
}

struct Nbr {
    int ox[5], oy[5], oz[5];  // element offsets for displacement d = -2..2 (index d + 2)
    __device__ __forceinline__ int at(int dx, int dy, int dz) const { return ox[dx + 2] + oy[dy + 2] + oz[dz + 2]; }
};

// STATE: offsets into the state arrays, which hold the ghost planes of a
// driven face below z = 0; otherwise offsets into plain N-cell field arrays
// (a driven face then acts as open).
template <bool STATE>
__device__ __forceinline__ Nbr make_nbr(const Consts& K, int x, int y, int z) {
    Nbr n;
    const int sy = K.nx, sz = K.nx * K.ny;
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        n.ox[d + 2] = map_coord(x + d, K.nx, K.per[0], 0) - x;
        n.oy[d + 2] = (map_coord(y + d, K.ny, K.per[1], 0) - y) * sy;
        n.oz[d + 2] = (map_coord(z + d, K.nz, K.per[2], STATE ? K.drv : 0) - z) * sz;
    }
    return n;
}

// Derivative along `axis` of a quantity X(x, y, z) at a cell: central
// differences (periodic wrap on periodic axes), one-sided towards the
// interior on the faces of a non-periodic axis, zero on an axis of one cell.
// The divergence operator of the normal-B adjustment and of max |div B|.
template <typename Fn>
__device__ __forceinline__ double axis_derivative(const Consts& K, int axis, int x, int y, int z, Fn&& X) {
    const int n = axis == 0 ? K.nx : (axis == 1 ? K.ny : K.nz);
    const int v = axis == 0 ? x : (axis == 1 ? y : z);
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    if (n == 1) return 0.0;
    if (!K.per[axis] && v == 0) return (X(x + ex, y + ey, z + ez) - X(x, y, z)) / K.dx;
    if (!K.per[axis] && v == n - 1) return (X(x, y, z) - X(x - ex, y - ey, z - ez)) / K.dx;
    const int wp = map_coord(v + 1, n, K.per[axis], 0) - v, wm = map_coord(v - 1, n, K.per[axis], 0) - v;
    return (X(x + ex * wp, y + ey * wp, z + ez * wp) - X(x + ex * wm, y + ey * wm, z + ez * wm)) / (2.0 * K.dx);
}

// Index of a face cell in the adjusted-normal-B arrays (face f = 2 axis + high).
__device__ __forceinline__ int64_t face_slot(const Consts& K, int f, int x, int y, int z) {
    const int a = f >> 1;
    const int64_t j = a == 0 ? y + (int64_t)K.ny * z : (a == 1 ? x + (int64_t)K.nx * z : x + (int64_t)K.nx * y);
    return K.fo[f] + j;
}

// Whether a cell lies on a face of a non-periodic axis other than `a` (an
// edge or corner cell when it also lies on a face of `a`).
__device__ __forceinline__ bool on_other_face(const Consts& K, int a, int x, int y, int z) {
    const int pos[3] = {x, y, z}, dims[3] = {K.nx, K.ny, K.nz};
    bool e = false;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (b != a && dims[b] >= 2 && !K.per[b] && (pos[b] == 0 || pos[b] == dims[b] - 1)) e = true;
    return e;
}

// Normal-B adjustment of an open-face cell (Sec. IV, KH set-up): on a face
// cell that is not an edge or corner cell, replace the normal component by
// the value the face pass computed.
__device__ __forceinline__ void apply_face_b(const Consts& K, const double* __restrict__ faceB, int x, int y, int z,
                                             double B[3]) {
    const int pos[3] = {x, y, z}, dims[3] = {K.nx, K.ny, K.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool lo = pos[a] == 0 && K.open_lo[a], hi = pos[a] == dims[a] - 1 && K.open_hi[a];
        if ((lo || hi) && !on_other_face(K, a, x, y, z)) B[a] = faceB[face_slot(K, lo ? 2 * a : 2 * a + 1, x, y, z)];
    }
}

// Tile index with XCD-aware placement: block b runs on XCD b % 8, so XCD k is
// given the contiguous tile range [k P, (k + 1) P).
__device__ __forceinline__ int tile_of_block(int nblocks) {
    const int P = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * P + blockIdx.x / 8;
}

// Moments and macroscopic solution of one cell in one step.
struct CellSol {
    double T00, T0[3], Tab[6], N0;   // moments (Tab: xx, yy, zz, xy, xz, yz)
    double Ep[3], B[3], rho, rho_g;  // previous E, this step's B, charge, Gauss charge
    double Epr[3];                   // E' of Eq. Cal_E
    double eps, p, n, gam, beta[3], E[3], J[3];
    int iters;
    int fallback;  // the learned guess was rejected (Newton started from E_f)
    bool ok;
};

// ... plus the transported f, g and streamed h (one thread per cell).
struct Macro : CellSol {
    double F[Q], G[Q], H[QH + 1];
};

// Fluid tensor T_fl = T - T_EM of the recovery: E_f = T_fl^00, S = T_fl^0a,
// Pi = T_fl^ab (xx, yy, zz, xy, xz, yz), with E_prev and the recovery's B
// (this step's, or with the previous-B reading the previous step's).
__device__ __forceinline__ void fluid_tensor(const Consts& K, const CellSol& M, const double (&B)[3], double& Ef,
                                             double S[3], double Pi[6]) {
    const double c = K.c, c2 = c * c;
    const double* E = M.Ep;
    const double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    const double U = 0.5 * (E2 + c2 * B2);
    Ef = M.T00 - K.eps0 * U;
    S[0] = M.T0[0] - K.eps0 * c * (E[1] * B[2] - E[2] * B[1]);
    S[1] = M.T0[1] - K.eps0 * c * (E[2] * B[0] - E[0] * B[2]);
    S[2] = M.T0[2] - K.eps0 * c * (E[0] * B[1] - E[1] * B[0]);
    Pi[0] = M.Tab[0] - K.eps0 * (U - E[0] * E[0] - c2 * B[0] * B[0]);
    Pi[1] = M.Tab[1] - K.eps0 * (U - E[1] * E[1] - c2 * B[1] * B[1]);
    Pi[2] = M.Tab[2] - K.eps0 * (U - E[2] * E[2] - c2 * B[2] * B[2]);
    Pi[3] = M.Tab[3] + K.eps0 * (E[0] * E[1] + c2 * B[0] * B[1]);
    Pi[4] = M.Tab[4] + K.eps0 * (E[0] * E[2] + c2 * B[0] * B[2]);
    Pi[5] = M.Tab[5] + K.eps0 * (E[1] * E[2] + c2 * B[1] * B[2]);
}

// Where the learned guess comes from: none (Newton from E_f), or the
// network evaluated on the wavefront with two lanes per cell (PAIR) or one
// lane per cell (SINGLE, two passes of 32 cells); MONITOR: Newton from E_f in
// a step with the guess enabled whose gate is closed, recording whether the
// gate opens for the next step.
enum GuessMode { GUESS_NONE = 0, GUESS_PAIR = 1, GUESS_SINGLE = 2, GUESS_MONITOR = 3 };

// Below this flow ratio |S| / E_f a cell takes no guess (Newton from E_f needs
// at most a few steps there, and on the flare box the network saved none for
// cells between 0.02 and 0.1), a wavefront of only such cells skips the
// network, and a step that meets no other cell closes the gate for the next.
#ifndef RMHDLB_GUESS_MIN_FLOW
#define RMHDLB_GUESS_MIN_FLOW 0.1
#endif
constexpr double GUESS_MIN_FLOW = RMHDLB_GUESS_MIN_FLOW;

// Record that this step met a cell above the gate (the lowest such lane of the
// wavefront stores; skipped once the slot holds this step's number).  Lanes
// that left the wavefront early do not take part.
__device__ __forceinline__ void open_gate(const Consts& K, bool moving) {
    const uint64_t m = __ballot(moving);
    if (K.gflag_wr && m && (int)(threadIdx.x & 63) == __builtin_ctzll(m) && *K.gflag_wr != K.gstep)
        *K.gflag_wr = K.gstep;
}

// Network guess of the eigenvalue for this lane's cell (all lanes of the
// wavefront call it together).  E_f (no guess) for nearly resting cells; NaN
// when the predicted |beta| >= 0.999 (those cells fall back to E_f).
template <int GM>
__device__ __forceinline__ double guess_lambda(const GuessTables* __restrict__ gt, double Ef, const double S[3],
                                               const double Pi[6], double N0, bool* gate) {
    double f[6], s;
    f[0] = flow_ratio(Ef, S, s);
    const bool moving = f[0] > GUESS_MIN_FLOW;
    if (!__any(moving)) return Ef;  // uniform over the wavefront
    if (gate) *gate = true;
    mlp_features(Ef, S, Pi, N0, s, f);
    float x[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = (float)((f[j] - (double)gt->mu_x[j]) * (double)gt->inv_sd_x[j]);
    const int lane = threadIdx.x & 63;
    float y0, y1;
    if constexpr (GM == GUESS_PAIR) {
        mlp_wave(gt, x, lane & 31, lane & 31, y0, y1);  // cell n of the wavefront is lane n (and n + 32)
    } else {
        float a0, a1, c0, c1;
        mlp_wave(gt, x, lane & 31, lane & 31, a0, a1);
        mlp_wave(gt, x, 32 + (lane & 31), lane & 31, c0, c1);
        y0 = lane < 32 ? a0 : c0;
        y1 = lane < 32 ? a1 : c1;
    }
    const double t0 = (double)gt->mu_t[0] + (double)gt->sd_t[0] * (double)y0;
    const double bn = (double)gt->mu_t[1] + (double)gt->sd_t[1] * (double)y1;
    if (!moving) return Ef;
    return bn < 0.999 ? Ef * t0 : __builtin_nan("");
}

// Recovery and the Ohm-coupled E, J of one cell from its moments (M.T00,
// M.T0, M.Tab, M.N0, M.Epr, M.B, M.Ep, M.rho_g): fills eps, p, n, gam, beta,
// E, J, iters, fallback, ok.  Brec is the B of the recovery's T_EM (M.B, or
// the previous step's B); the Ohm solve always takes M.B.  With a guess mode
// every lane of the wavefront must call it together, and *gate (when given,
// uniform over the wavefront) is set when a cell of the wavefront lies above
// the guess's flow-ratio gate.
template <int GM = GUESS_NONE>
__device__ __forceinline__ void solve_cell(const Consts& K, CellSol& M, const double (&Brec)[3],
                                           const GuessTables* __restrict__ gt = nullptr, bool* gate = nullptr) {
    const double c = K.c, c2 = c * c;
    const double* B = M.B;
    double Ef, S[3], Pi[6];
    fluid_tensor(K, M, Brec, Ef, S, Pi);
    double lam;
    if constexpr (GM == GUESS_MONITOR)
        if (gate && __any(S[0] * S[0] + S[1] * S[1] + S[2] * S[2] > (GUESS_MIN_FLOW * Ef) * (GUESS_MIN_FLOW * Ef)))
            *gate = true;
    if constexpr (GM == GUESS_NONE || GM == GUESS_MONITOR) {
        M.iters = recover(Ef, S, Pi, lam, M.beta);
        M.fallback = 0;
    } else {
        const double lam0 = guess_lambda<GM>(gt, Ef, S, Pi, M.N0, gate);
        M.iters = recover_from_guess(Ef, S, Pi, lam0, lam, M.beta, M.fallback);
    }
    const double b2 = M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] + M.beta[2] * M.beta[2];
    M.gam = 1.0 / sqrt(1.0 - b2);
    M.n = M.N0 / M.gam;
    M.p = K.gm1 * (lam - M.n * c2);
    M.eps = lam;
    M.ok = (b2 < 1.0) && (lam > 0.0) && (M.n > 0.0) && (M.p >= 0.0) && isfinite(M.p);
    if (!M.ok) {
        const double nan = __builtin_nan("");
        M.eps = M.p = M.n = M.gam = nan;
#pragma unroll
        for (int a = 0; a < 3; ++a) M.beta[a] = M.E[a] = M.J[a] = nan;
        return;
    }

    // E from E = E' - (dt/2) mu0 c^2 J(E) with Eq. Ohm, by Sherman-Morrison:
    // (1 + K) E - (K / c^2)(E.u) u = R, R = E' - K u x B - q rho_G u
    const double u0 = c * M.beta[0], u1 = c * M.beta[1], u2 = c * M.beta[2];
    const double Kf = K.q * K.sigma * M.gam;
    const double uxB0 = u1 * B[2] - u2 * B[1], uxB1 = u2 * B[0] - u0 * B[2], uxB2 = u0 * B[1] - u1 * B[0];
    const double qr = K.q * M.rho_g;
    const double R0 = M.Epr[0] - Kf * uxB0 - qr * u0;
    const double R1 = M.Epr[1] - Kf * uxB1 - qr * u1;
    const double R2 = M.Epr[2] - Kf * uxB2 - qr * u2;
    const double uR = u0 * R0 + u1 * R1 + u2 * R2;
    const double coef = (Kf / c2) * uR / (1.0 + Kf * (1.0 - b2));
    const double inv1K = 1.0 / (1.0 + Kf);
    M.E[0] = (R0 + coef * u0) * inv1K;
    M.E[1] = (R1 + coef * u1) * inv1K;
    M.E[2] = (R2 + coef * u2) * inv1K;
    const double Eu = (M.E[0] * u0 + M.E[1] * u1 + M.E[2] * u2) / c2;
    const double sg = K.sigma * M.gam;
    M.J[0] = sg * (M.E[0] + uxB0 - Eu * u0) + M.rho_g * u0;
    M.J[1] = sg * (M.E[1] + uxB1 - Eu * u1) + M.rho_g * u1;
    M.J[2] = sg * (M.E[2] + uxB2 - Eu * u2) + M.rho_g * u2;
}

// Transport (collide-then-transport reading of Eq. rlb): link-wise
// minmod-MUSCL flux difference, plus the 7-point bulk-viscosity Laplacian
// for i != 0; g without viscosity.  Then the streaming of h, the moments,
// the recovery and E, J.
// One thread per cell, FP64 arithmetic (moments and diagnostics pass).  The
// shift of a stored array is constant in space, so it transports to itself
// and is added back after the transport.
template <int GM, typename TS, typename TE>
__device__ __forceinline__ void macroscopic(const TS* __restrict__ src, const TE* __restrict__ esrc,
                                            const double* __restrict__ faceB, const GuessTables* __restrict__ gt,
                                            const Consts& K, int cell, const Nbr& nb, int x, int y, int z, Macro& M) {
    M.T00 = 0.0;
    M.N0 = 0.0;
    double t0x = 0, t0y = 0, t0z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        auto fg = [&](int o) {
            vec2<double> r;
            r.x = ld(src, f_at<TS>(K, i, (int64_t)cell + o));
            r.y = ld(src, g_at<TS>(K, i, (int64_t)cell + o));
            return r;
        };
        auto fo = [&](int o) { return ld(src, f_at<TS>(K, i, (int64_t)cell + o)); };
        const vec2<double> c0 = fg(0);
        const double f0 = c0.x, g0 = c0.y;
        double fv = f0, gv = g0;
        if (i != 0) {
            const int ex = EX[i], ey = EY[i], ez = EZ[i];
            const int om2 = nb.at(-2 * ex, -2 * ey, -2 * ez), om1 = nb.at(-ex, -ey, -ez), op1 = nb.at(ex, ey, ez);
            const vec2<double> m2 = fg(om2), m1 = fg(om1), p1 = fg(op1);
            {
                const double fm2 = m2.x, fm1 = m1.x, fp1 = p1.x;
                const double face_p = f0 + K.slope * minmod(f0 - fm1, fp1 - f0);
                const double face_m = fm1 + K.slope * minmod(fm1 - fm2, f0 - fm1);
                const double lap = (fo(nb.at(1, 0, 0)) + fo(nb.at(-1, 0, 0))) +
                                   (fo(nb.at(0, 1, 0)) + fo(nb.at(0, -1, 0))) +
                                   (fo(nb.at(0, 0, 1)) + fo(nb.at(0, 0, -1))) - 6.0 * f0;
                fv = f0 - K.cour * (face_p - face_m) + K.kv * lap;
            }
            {
                const double gm2 = m2.y, gm1 = m1.y, gp1 = p1.y;
                const double face_p = g0 + K.slope * minmod(g0 - gm1, gp1 - g0);
                const double face_m = gm1 + K.slope * minmod(gm1 - gm2, g0 - gm1);
                gv = g0 - K.cour * (face_p - face_m);
            }
        }
        fv += fshift(K, i);
        gv += gshift(K, i);
        M.F[i] = fv;
        M.G[i] = gv;
        M.T00 += fv;
        M.N0 += gv;
        if (EX[i]) t0x += EX[i] * fv;
        if (EY[i]) t0y += EY[i] * fv;
        if (EZ[i]) t0z += EZ[i] * fv;
        if (EX[i]) txx += fv;
        if (EY[i]) tyy += fv;
        if (EZ[i]) tzz += fv;
        if (EX[i] * EY[i]) txy += (EX[i] * EY[i]) * fv;
        if (EX[i] * EZ[i]) txz += (EX[i] * EZ[i]) * fv;
        if (EY[i] * EZ[i]) tyz += (EY[i] * EZ[i]) * fv;
    }
    M.T0[0] = KAPPA * t0x;
    M.T0[1] = KAPPA * t0y;
    M.T0[2] = KAPPA * t0z;
    M.Tab[0] = KAPPA2 * txx;
    M.Tab[1] = KAPPA2 * tyy;
    M.Tab[2] = KAPPA2 * tzz;
    M.Tab[3] = KAPPA2 * txy;
    M.Tab[4] = KAPPA2 * txz;
    M.Tab[5] = KAPPA2 * tyz;

    // stream h (Eq. LB_Maxwell): h_k(x) = h*_k(x - v_k dt)
    double ehx = 0, ehy = 0, ehz = 0, bx = 0, by = 0, bz = 0, hs = 0;
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const double h = ld(src, h_at<TS>(K, k, (int64_t)cell + nb.at(-SX[k], -SY[k], -SZ[k])));
        M.H[k] = h;
        hs += h;
        if (EHX[k]) ehx += EHX[k] * h;
        if (EHY[k]) ehy += EHY[k] * h;
        if (EHZ[k]) ehz += EHZ[k] * h;
        if (BHX[k]) bx += BHX[k] * h;
        if (BHY[k]) by += BHY[k] * h;
        if (BHZ[k]) bz += BHZ[k] * h;
    }
    M.H[QH] = ld(src, h_at<TS>(K, QH, cell));
    const double ec = K.c * INV_SQRT2;  // |e_k| / |ehat_k|
    M.Epr[0] = ec * ehx;
    M.Epr[1] = ec * ehy;
    M.Epr[2] = ec * ehz;
    M.B[0] = bx;
    M.B[1] = by;
    M.B[2] = bz;
    M.rho = M.H[QH] + hs;

    // previous E and its Gauss charge
    const TE* __restrict__ e0 = esrc + cell;
    const TE* __restrict__ e1 = esrc + K.stride + cell;
    const TE* __restrict__ e2 = esrc + 2 * K.stride + cell;
    M.Ep[0] = ld(e0, 0);
    M.Ep[1] = ld(e1, 0);
    M.Ep[2] = ld(e2, 0);
    M.rho_g = K.eps0 * K.inv_2dx *
              ((ld(e0, nb.at(1, 0, 0)) - ld(e0, nb.at(-1, 0, 0))) + (ld(e1, nb.at(0, 1, 0)) - ld(e1, nb.at(0, -1, 0))) +
               (ld(e2, nb.at(0, 0, 1)) - ld(e2, nb.at(0, 0, -1))));

    if (K.divb) apply_face_b(K, faceB, x, y, z, M.B);
    if (K.bprev) {
        double Bp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Bp[a] = ld(esrc + (int64_t)(3 + a) * K.stride + cell, 0);
        solve_cell<GM>(K, M, Bp, gt);
    } else {
        solve_cell<GM>(K, M, M.B, gt);
    }
}

// f_eq of Eq. Dis_fun_EM in normalised variables (F = (c_t/c_0)^2 f), with
// the corrections that make its moments T_fluid + T_EM: the delta_i0
// coefficient 361 (3p - eps) / (33 (p + eps)), the minus sign of the
// (E.c_i)^2 term, the y-z cross terms, and c on the (B x E).c_i term.
// The per-cell setup runs in FP64; the per-direction evaluation in V (FP64 on
// the plain path, FP32 on the mixed-storage paths).
template <typename V>
struct FeqCellT {
    V P34, A1, Bc, g2, beta[3], b2, eps0;
    V X, BxE[3], E[3], cB[3];
    __device__ __forceinline__ void setup(double eps, double p, double gam, const double bta[3], const double Ev[3],
                                          const double Bv[3], double c, double e0) {
        P34 = (V)(0.75 * (eps + p));
        A1 = (V)(1.0 + (3.0 * p - eps) / (p + eps));
        Bc = (V)(361.0 * (3.0 * p - eps) / (33.0 * (p + eps)));
        g2 = (V)(gam * gam);
        b2 = (V)(bta[0] * bta[0] + bta[1] * bta[1] + bta[2] * bta[2]);
        double cb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            beta[a] = (V)bta[a];
            E[a] = (V)Ev[a];
            cb[a] = c * Bv[a];
            cB[a] = (V)cb[a];
        }
        X = (V)(cb[0] * cb[0] + cb[1] * cb[1] + cb[2] * cb[2] + Ev[0] * Ev[0] + Ev[1] * Ev[1] + Ev[2] * Ev[2]);
        // c (B x E)
        BxE[0] = (V)(cb[1] * Ev[2] - cb[2] * Ev[1]);
        BxE[1] = (V)(cb[2] * Ev[0] - cb[0] * Ev[2]);
        BxE[2] = (V)(cb[0] * Ev[1] - cb[1] * Ev[0]);
        eps0 = (V)e0;
    }
    template <int I>
    __device__ __forceinline__ V eq() const {
        constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
        const V eb = ex * beta[0] + ey * beta[1] + ez * beta[2];
        const V cross = (ex * ey) * beta[0] * beta[1] + (ex * ez) * beta[0] * beta[2] + (ey * ez) * beta[1] * beta[2];
        const V diag = (ex * ex) * beta[0] * beta[0] + (ey * ey) * beta[1] * beta[1] + (ez * ez) * beta[2] * beta[2];
        V fluid = A1 + V(19) * g2 * cross + V(4 * KAPPA) * g2 * eb + V(4.0 / 15.0) * g2 * (V(19) * diag - V(4) * b2);
        if (I == 0) fluid += Bc;
        const V Be = ex * cB[0] + ey * cB[1] + ez * cB[2];
        const V Ee = ex * E[0] + ey * E[1] + ez * E[2];
        const V BxEe = ex * BxE[0] + ey * BxE[1] + ez * BxE[2];
        const V crossEB = (ex * ey) * (E[0] * E[1] + cB[0] * cB[1]) + (ex * ez) * (E[0] * E[2] + cB[0] * cB[2]) +
                          (ey * ez) * (E[1] * E[2] + cB[1] * cB[2]);
        const V em = V(2.3) * X - V(SQRT19_3) * BxEe - V(3.8) * (Be * Be + Ee * Ee) - V(6.65) * crossEB;
        return V(weight(I)) * (P34 * fluid + eps0 * em);
    }
};
using FeqCell = FeqCellT<double>;

// f_eq of direction sgn * e_I (sgn = +-1): the odd terms change sign, the
// weight is that of e_I.
template <int I, typename V>
__device__ __forceinline__ V feq_signed(const FeqCellT<V>& f, V sgn) {
    constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
    const V eb = sgn * (ex * f.beta[0] + ey * f.beta[1] + ez * f.beta[2]);
    const V cross =
        (ex * ey) * f.beta[0] * f.beta[1] + (ex * ez) * f.beta[0] * f.beta[2] + (ey * ez) * f.beta[1] * f.beta[2];
    const V diag = (ex * ex) * f.beta[0] * f.beta[0] + (ey * ey) * f.beta[1] * f.beta[1] +
                   (ez * ez) * f.beta[2] * f.beta[2];
    const V fluid =
        f.A1 + V(19) * f.g2 * cross + V(4 * KAPPA) * f.g2 * eb + V(4.0 / 15.0) * f.g2 * (V(19) * diag - V(4) * f.b2);
    const V Be = ex * f.cB[0] + ey * f.cB[1] + ez * f.cB[2];
    const V Ee = ex * f.E[0] + ey * f.E[1] + ez * f.E[2];
    const V BxEe = sgn * (ex * f.BxE[0] + ey * f.BxE[1] + ez * f.BxE[2]);
    const V crossEB = (ex * ey) * (f.E[0] * f.E[1] + f.cB[0] * f.cB[1]) +
                      (ex * ez) * (f.E[0] * f.E[2] + f.cB[0] * f.cB[2]) +
                      (ey * ez) * (f.E[1] * f.E[2] + f.cB[1] * f.cB[2]);
    const V em = V(2.3) * f.X - V(SQRT19_3) * BxEe - V(3.8) * (Be * Be + Ee * Ee) - V(6.65) * crossEB;
    return V(weight(I)) * (f.P34 * fluid + f.eps0 * em);
}

template <int I, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    if constexpr (I < Q) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1>(fn);
    }
}

// ---------------------------------------------------- two lanes per cell

// The fused step with the populations of one cell split over a lane pair
// (lanes l and l ^ 32 of a wavefront, h = 0, 1).  Slot s = 1..9 of f and g is direction 2s-1+h,
// i.e. sgn * e_{2s-1} with sgn = +1 / -1, so both lanes run the same
// instructions on opposite directions; slot m = 0..11 of h is population
// 2m+h (same streaming offset, opposite e and b).  Lane 0 also owns the rest
// populations f_0, g_0; lane 1 owns h_rest.  Partial moments are summed over
// the pair with one xor-32 shuffle each, and both lanes then run the recovery
// and the Ohm solve on identical inputs.
//
// f and g are handled as stored deviations d (the shift is 0 on the plain
// path): the transport is linear and the shift is uniform, so the transported
// value is shift + transport(d); the moments add the exact sums of the shifts;
// the collisions write the new deviations directly.
constexpr int PTPB = 256;  // threads of a fused-step block: 128 cells, two lanes each
// Waves per SIMD the fused kernel is compiled for: two for the FP64 and
// FP32 forms (they lose more to spills at three than they gain: FP32 4 %
// slower), three for FP16 storage (plain FP16 3.6 % faster on the flare box
// than two and 31 % faster than four; with the learned guess, once the lane
// coordinates are recomputed per plane, 2.5 % faster than two).
#ifndef RMHDLB_WAVES
#define RMHDLB_WAVES 2
#endif
#ifndef RMHDLB_WAVES_F16
#define RMHDLB_WAVES_F16 2
#endif
template <typename TS, int GM>
constexpr int fused_waves() {
    return sizeof(TS) == 2 ? RMHDLB_WAVES_F16 : RMHDLB_WAVES;
}
// f/g slots whose loads may be in flight together, per storage type
// (measured on the flare box: 2 for FP64, where 1 is 18 % and 3 is 25 %
// slower; 3 for FP32, where 2 is 4 % and 4 is 8 % slower; 3 for FP16, 1.5 %
// faster than 2 with and without the guess, and 1-2 % faster than 4, 5, 9)
#ifndef RMHDLB_GROUP_F64
#define RMHDLB_GROUP_F64 2
#endif
#ifndef RMHDLB_GROUP_F32
#define RMHDLB_GROUP_F32 3
#endif
#ifndef RMHDLB_GROUP_F16
#define RMHDLB_GROUP_F16 3
#endif
template <typename TS>
constexpr int pin_group() {
    return sizeof(TS) == 8 ? RMHDLB_GROUP_F64 : (sizeof(TS) == 4 ? RMHDLB_GROUP_F32 : RMHDLB_GROUP_F16);
}

// The two lanes of a cell are l and l ^ 32 of a wavefront: each half of the
// wavefront then reads 32 consecutive values of one array, which the vector
// memory path coalesces (with the partner in the adjacent lane every
// instruction touched two arrays lane by lane and the texture units, not
// HBM, set the step time).
template <typename V>
__device__ __forceinline__ V pair_sum(V v) {
    return v + __shfl_xor(v, 32, 64);
}

// VR: the alternative readings, bit 0 the printed semi-implicit f collision
// of Eq. rlb, f' = (f + omega f_eq) / (1 + omega) (else explicit, Reading
// R4); bit 1 the limited Lax-Wendroff face values (else MUSCL, Reading R2);
// bit 2 the external force; bit 3 the previous step's B in the recovery and
// f_eq (else this step's, Reading R10), carried in the field block.
template <bool NT, typename TS, typename TE, typename V, int GM, int VR = 0>
__device__ __forceinline__ void pair_cell(const TS* __restrict__ sd, const TE* __restrict__ se, TS* __restrict__ dd,
                                          TE* __restrict__ de, const double* __restrict__ faceB,
                                          const GuessTables* __restrict__ gt, const Consts& K, int cell,
                                          const Nbr& nb, int h, int x, int y, int z, bool active, double& bmax,
                                          bool& gate) {
    // stores of this cell's new state (lanes that only take part in the
    // wavefront's network evaluation store nothing)
    auto put = [&](auto* p, auto v) {
        if (active) st<NT>(p, v);
    };
    const V sgn = h ? V(-1) : V(1);
    const int64_t S = K.stride;
    // Array bases stay uniform (scalar registers); the lane's choice between
    // the two arrays of a pair is folded into its 32-bit element index.
    const int hc = cell + (h ? (int)S : 0);
    constexpr int CM = VR & 1;
    const V cour = (V)K.cour, kv = (V)K.kv, slope = (VR & 2) ? (V)K.slope : V(0.5);
    V Fv[10], Gv[10], Hv[13];
    V t00 = 0, t0x = 0, t0y = 0, t0z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0, n0 = 0;
    // slot 0: f_0, g_0 (lane 0) and h_rest (lane 1)
    {
        const vec2<V> fg0 = ldv2<V>(sd, fg_index(K, 0, cell));
        const V hr = ldv_once<V>(sd, (int64_t)(OFF_H + QH) * S + cell);
        Fv[0] = h ? V(0) : fg0.x;
        Gv[0] = h ? V(0) : fg0.y;
        Hv[12] = h ? hr : V(0);
        t00 = Fv[0];
        n0 = Gv[0];
    }
    const int lap_xp = nb.at(1, 0, 0), lap_xm = nb.at(-1, 0, 0), lap_yp = nb.at(0, 1, 0), lap_ym = nb.at(0, -1, 0),
              lap_zp = nb.at(0, 0, 1), lap_zm = nb.at(0, 0, -1);
    static_for<1>([&](auto ic) {
        constexpr int s = decltype(ic)::value;
        if constexpr (s <= 9) {
            constexpr int i0 = 2 * s - 1;
            constexpr int ex = EX[i0], ey = EY[i0], ez = EZ[i0];
            const int om2 = h ? nb.at(2 * ex, 2 * ey, 2 * ez) : nb.at(-2 * ex, -2 * ey, -2 * ez);
            const int om1 = h ? nb.at(ex, ey, ez) : nb.at(-ex, -ey, -ez);
            const int op1 = h ? nb.at(-ex, -ey, -ez) : nb.at(ex, ey, ez);
            const TS* __restrict__ fga = sd + fg_index(K, i0, 0);  // uniform base of direction i0's pairs
            const vec2<V> c0 = ldv2<V>(fga, 2 * (int64_t)hc), m2 = ldv2<V>(fga, 2 * (int64_t)(hc + om2)),
                          m1 = ldv2<V>(fga, 2 * (int64_t)(hc + om1)), p1 = ldv2<V>(fga, 2 * (int64_t)(hc + op1));
            const V f0 = c0.x, fm2 = m2.x, fm1 = m1.x, fp1 = p1.x;
            // On an axis slot the upwind points x -+ e are also the Laplacian's
            // neighbours along that axis (lane 1 walks -e): reuse them.
            constexpr bool axis_slot = (ex != 0) + (ey != 0) + (ez != 0) == 1;
            const V up = h ? fm1 : fp1, dn = h ? fp1 : fm1;  // f at x + e_i0 and x - e_i0
            auto lap_at = [&](int off) { return ldv<V>(fga, 2 * (int64_t)(hc + off)); };
            V lxp, lxm, lyp, lym, lzp, lzm;
            if constexpr (axis_slot && ex != 0) {
                lxp = up;
                lxm = dn;
            } else {
                lxp = lap_at(lap_xp);
                lxm = lap_at(lap_xm);
            }
            if constexpr (axis_slot && ey != 0) {
                lyp = up;
                lym = dn;
            } else {
                lyp = lap_at(lap_yp);
                lym = lap_at(lap_ym);
            }
            if constexpr (axis_slot && ez != 0) {
                lzp = up;
                lzm = dn;
            } else {
                lzp = lap_at(lap_zp);
                lzm = lap_at(lap_zm);
            }
            const V lap = (lxp + lxm) + (lyp + lym) + (lzp + lzm) - V(6) * f0;
            const V fv = f0 - cour * ((f0 + slope * minmod(f0 - fm1, fp1 - f0)) -
                                      (fm1 + slope * minmod(fm1 - fm2, f0 - fm1))) + kv * lap;
            const V g0 = c0.y, gm2 = m2.y, gm1 = m1.y, gp1 = p1.y;
            const V gv = g0 - cour * ((g0 + slope * minmod(g0 - gm1, gp1 - g0)) -
                                      (gm1 + slope * minmod(gm1 - gm2, g0 - gm1)));
            Fv[s] = fv;
            Gv[s] = gv;
            // Keep each slot's arithmetic next to its loads: without this the
            // scheduler sinks all of it below every load of the cell, and the
            // ~150 load destinations in flight cost a wave its occupancy.
            if constexpr (s % pin_group<TS>() == 0 || s == 9) asm volatile("" : "+v"(Fv[s]), "+v"(Gv[s])::"memory");
            t00 += fv;
            n0 += gv;
            const V sf = sgn * fv;
            if (ex) t0x += ex * sf;
            if (ey) t0y += ey * sf;
            if (ez) t0z += ez * sf;
            if (ex) txx += fv;
            if (ey) tyy += fv;
            if (ez) tzz += fv;
            if (ex * ey) txy += (ex * ey) * fv;
            if (ex * ez) txz += (ex * ez) * fv;
            if (ey * ez) tyz += (ey * ez) * fv;
        }
    });
    V ehx = 0, ehy = 0, ehz = 0, bx = 0, by = 0, bz = 0, hs = 0;
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const V v = ldv_once<V>(sd + (int64_t)(OFF_H + k0) * S, hc + nb.at(-SX[k0], -SY[k0], -SZ[k0]));
        Hv[m] = v;
        hs += v;
        const V sv = sgn * v;
        if (EHX[k0]) ehx += EHX[k0] * sv;
        if (EHY[k0]) ehy += EHY[k0] * sv;
        if (EHZ[k0]) ehz += EHZ[k0] * sv;
        if (BHX[k0]) bx += BHX[k0] * sv;
        if (BHY[k0]) by += BHY[k0] * sv;
        if (BHZ[k0]) bz += BHZ[k0] * sv;
    }
    CellSol M;
#pragma unroll
    for (int a = 0; a < 3; ++a) M.Ep[a] = ld(se + (int64_t)a * S + cell, 0);
    // Gauss charge: lane 0 takes E_x(x+-1), E_y(y+1); lane 1 E_y(y-1), E_z(z+-1)
    double gpart;
    {
        const TE* ex_ = se + cell;
        const TE* ey_ = se + S + cell;
        const TE* ez_ = se + 2 * S + cell;
        const double a = h ? -ld(ey_, lap_ym) : ld(ex_, lap_xp);
        const double b = h ? ld(ez_, lap_zp) : -ld(ex_, lap_xm);
        const double c = h ? -ld(ez_, lap_zm) : ld(ey_, lap_yp);
        gpart = (a + b) + c;
    }
    M.T00 = K.fs0 + (double)pair_sum(t00);
    M.N0 = K.gs0 + (double)pair_sum(n0);
    M.T0[0] = KAPPA * (double)pair_sum(t0x);
    M.T0[1] = KAPPA * (double)pair_sum(t0y);
    M.T0[2] = KAPPA * (double)pair_sum(t0z);
    M.Tab[0] = KAPPA2 * (K.fsaa + (double)pair_sum(txx));
    M.Tab[1] = KAPPA2 * (K.fsaa + (double)pair_sum(tyy));
    M.Tab[2] = KAPPA2 * (K.fsaa + (double)pair_sum(tzz));
    M.Tab[3] = KAPPA2 * (double)pair_sum(txy);
    M.Tab[4] = KAPPA2 * (double)pair_sum(txz);
    M.Tab[5] = KAPPA2 * (double)pair_sum(tyz);
    const double ec = K.c * INV_SQRT2;
    M.Epr[0] = ec * (double)pair_sum(ehx);
    M.Epr[1] = ec * (double)pair_sum(ehy);
    M.Epr[2] = ec * (double)pair_sum(ehz);
    M.B[0] = (double)pair_sum(bx);
    M.B[1] = (double)pair_sum(by);
    M.B[2] = (double)pair_sum(bz);
    // The Maxwell populations relax towards h_eq of the streamed B (an
    // adjusted face B enters only the fluid coupling): take its B part,
    // B . b_k / 8, into h* = 2 h_eq - h now, while the streamed B is at hand.
    {
        const V sb0 = (V)M.B[0], sb1 = (V)M.B[1], sb2 = (V)M.B[2];
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const int k0 = 2 * m;
            Hv[m] -= V(0.25) * sgn * (BHX[k0] * sb0 + BHY[k0] * sb1 + BHZ[k0] * sb2);
        }
    }
    M.rho = (double)pair_sum(Hv[12] + hs);
    M.rho_g = K.eps0 * K.inv_2dx * pair_sum(gpart);
    if (K.divb) apply_face_b(K, faceB, x, y, z, M.B);
    FeqCellT<V> fe;
    if constexpr ((VR & 8) != 0) {
        double Bp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Bp[a] = ld(se + (int64_t)(3 + a) * S + cell, 0);
        solve_cell<GM>(K, M, Bp, gt, &gate);
        fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, Bp, K.c, K.eps0);
    } else {
        solve_cell<GM>(K, M, M.B, gt, &gate);
        fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, M.B, K.c, K.eps0);
    }

    // collisions and stores (new deviations)
    const V rate = (V)(M.gam * K.inv_tau);
    const V wg = (V)K.wg, inv1wg = (V)(1.0 / (1.0 + K.wg));
    const V ng = (V)(M.n * M.gam);
    const V gc1 = (V)K.gc1, gc2 = (V)K.gc2, gc3b2 = (V)(K.gc3 * (M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] +
                                                              M.beta[2] * M.beta[2]));
    const V bx_ = (V)M.beta[0], by_ = (V)M.beta[1], bz_ = (V)M.beta[2];
    // External force (Reading R26): c dt F^a into T^{0a} through the moving
    // populations, (19/9) w_i (e_i . c dt F) / kappa each, and the work
    // c dt F . beta into T^00 through the rest population; on while the
    // previous step's largest |beta| is below the gate.
    double fw = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if constexpr ((VR & 4) != 0) {
        bmax = fmax(bmax, sqrt(M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] + M.beta[2] * M.beta[2]));
        if (!(K.fgate > 0.0) || *K.vmax_prev < K.fgate) {
            const double cdt = K.dx * INV_SQRT2;  // c dt
            fx = cdt * K.force[cell];
            fy = cdt * K.force[K.N + cell];
            fz = cdt * K.force[2 * K.N + cell];
            fw = fx * M.beta[0] + fy * M.beta[1] + fz * M.beta[2];
        }
    }
    if (h == 0) {
        const V q0 = (V)K.fsh[0] - fe.template eq<0>();
        const V geq0 = (V)K.wp[0] * ng * (V(1) - gc3b2);
        V f0n = CM == 0 ? Fv[0] - rate * (Fv[0] + q0) : (Fv[0] - rate * q0) / (V(1) + rate);
        if constexpr ((VR & 4) != 0) f0n += (V)fw;
        if (active) st2<NT>(dd + fg_index(K, 0, cell), f0n, (Gv[0] + wg * (geq0 - (V)K.gsh[0])) * inv1wg);
    } else {
        put(dd + (int64_t)(OFF_H + QH) * S + cell, (V)(2.0 * M.rho) - Hv[12]);
    }
    static_for<1>([&](auto ic) {
        constexpr int s = decltype(ic)::value;
        if constexpr (s <= 9) {
            constexpr int i0 = 2 * s - 1;
            constexpr int cls = i0 <= 6 ? 1 : 2;
            const V eb = sgn * (EX[i0] * bx_ + EY[i0] * by_ + EZ[i0] * bz_);
            const V om = rate * (V(1) - V(KAPPA) * eb);
            const V q = (V)K.fsh[cls] - feq_signed<i0>(fe, sgn);
            const V geq = (V)K.wp[cls] * ng * (V(1) + gc1 * eb + gc2 * eb * eb - gc3b2);
            V fn = CM == 0 ? Fv[s] - om * (Fv[s] + q) : (Fv[s] - om * q) / (V(1) + om);
            if constexpr ((VR & 4) != 0) {
                constexpr double wcls = cls == 1 ? 99.0 / 722.0 : 9.0 / 361.0;  // D3Q19 weights
                fn += (V)((19.0 / 9.0) * wcls / KAPPA * ((h ? -1.0 : 1.0) * (EX[i0] * fx + EY[i0] * fy + EZ[i0] * fz)));
            }
            if (active)
                st2<NT>(dd + fg_index(K, i0, 0) + 2 * (int64_t)hc, fn, (Gv[s] + wg * (geq - (V)K.gsh[cls])) * inv1wg);
        }
    });
    const V cj = (V)(1.0 / (16.0 * 1.4142135623730951 * K.c)), ce = (V)(1.0 / (8.0 * 1.4142135623730951 * K.c));
    const V J0 = (V)M.J[0], J1 = (V)M.J[1], J2 = (V)M.J[2];
    const V E0 = (V)M.E[0], E1 = (V)M.E[1], E2 = (V)M.E[2];
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const V heq = cj * (SX[k0] * J0 + SY[k0] * J1 + SZ[k0] * J2) + sgn * ce * (EHX[k0] * E0 + EHY[k0] * E1 + EHZ[k0] * E2);
        put(dd + (int64_t)(OFF_H + k0) * S + hc, V(2) * heq - Hv[m]);
    }
    if (h == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) put(de + (int64_t)a * S + cell, M.E[a]);
    } else if constexpr ((VR & 8) != 0) {  // this step's coupling B is the next one's previous B
#pragma unroll
        for (int a = 0; a < 3; ++a) put(de + (int64_t)(3 + a) * S + cell, M.B[a]);
    }
}

// ---------------------------------------------------- one lane per cell

template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));

template <typename V, typename T>
__device__ __forceinline__ vec4<V> ldv4(const T* __restrict__ p, int64_t i) {
    const vec4<T> v = *reinterpret_cast<const vec4<T>*>(p + i);
    vec4<V> r;
    r.x = static_cast<V>(v.x);
    r.y = static_cast<V>(v.y);
    r.z = static_cast<V>(v.z);
    r.w = static_cast<V>(v.w);
    return r;
}

// 16 bytes of FP16 (two quads) at element i
template <typename V, typename T>
__device__ __forceinline__ void ldv8(const T* __restrict__ p, int64_t i, vec4<V>& lo, vec4<V>& hi) {
    typedef T vec8 __attribute__((ext_vector_type(8)));
    const vec8 v = *reinterpret_cast<const vec8*>(p + i);
    lo.x = static_cast<V>(v[0]);
    lo.y = static_cast<V>(v[1]);
    lo.z = static_cast<V>(v[2]);
    lo.w = static_cast<V>(v[3]);
    hi.x = static_cast<V>(v[4]);
    hi.y = static_cast<V>(v[5]);
    hi.z = static_cast<V>(v[6]);
    hi.w = static_cast<V>(v[7]);
}

template <bool NT, typename T, typename V>
__device__ __forceinline__ void st8(T* __restrict__ p, const vec4<V>& lo, const vec4<V>& hi) {
    typedef T vec8 __attribute__((ext_vector_type(8)));
    vec8 v;
    v[0] = static_cast<T>(lo.x);
    v[1] = static_cast<T>(lo.y);
    v[2] = static_cast<T>(lo.z);
    v[3] = static_cast<T>(lo.w);
    v[4] = static_cast<T>(hi.x);
    v[5] = static_cast<T>(hi.y);
    v[6] = static_cast<T>(hi.z);
    v[7] = static_cast<T>(hi.w);
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<vec8*>(p));
    else
        *reinterpret_cast<vec8*>(p) = v;
}

template <bool NT, typename T, typename V>
__device__ __forceinline__ void st4(T* __restrict__ p, V a, V b, V c, V d) {
    vec4<T> v;
    v.x = static_cast<T>(a);
    v.y = static_cast<T>(b);
    v.z = static_cast<T>(c);
    v.w = static_cast<T>(d);
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<vec4<T>*>(p));
    else
        *reinterpret_cast<vec4<T>*>(p) = v;
}

// f/g slots whose loads may be in flight together in the one-lane-per-cell step
#ifndef RMHDLB_QGROUP
#define RMHDLB_QGROUP 1
#endif

// The fused step of one cell in one lane (FP32 storage, quad layout; FP16,
// double-quad layout, where one load at the centre and at each Laplacian
// point serves the two slots of a record):
// slot s = 1..9 carries the opposite directions i0 = 2s - 1 (+e) and
// i1 = 2s (-e), and one load per point of the link x - 2e .. x + 2e and of the
// Laplacian serves both; the Maxwell populations 2m, 2m + 1 come from one load
// of the cell they stream from.  The arithmetic per direction is that of
// pair_cell (the readings it implements are listed there); only the
// assignment of work to lanes and the order of the moment sums differ.
template <bool NT, typename TS, typename TE, typename V, int GM, int VR = 0>
__device__ __forceinline__ void quad_cell(const TS* __restrict__ sd, const TE* __restrict__ se, TS* __restrict__ dd,
                                          TE* __restrict__ de, const double* __restrict__ faceB,
                                          const GuessTables* __restrict__ gt, const Consts& K, int cell,
                                          const Nbr& nb, int x, int y, int z, bool active, double& bmax,
                                          bool& gate) {
    auto put = [&](auto* p, auto v) {
        if (active) st<NT>(p, v);
    };
    const int64_t S = K.stride;
    constexpr int CM = VR & 1;
    const V cour = (V)K.cour, kv = (V)K.kv, slope = (VR & 2) ? (V)K.slope : V(0.5);
    V Fv[Q], Gv[Q], Hv[QH + 1];
    V t00 = 0, t0x = 0, t0y = 0, t0z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0, n0 = 0;
    const int lap_xp = nb.at(1, 0, 0), lap_xm = nb.at(-1, 0, 0), lap_yp = nb.at(0, 1, 0), lap_ym = nb.at(0, -1, 0),
              lap_zp = nb.at(0, 0, 1), lap_zm = nb.at(0, 0, -1);
    // Transport and moments of slot s from its quads at the link points x - 2e .. x + 2e and the
    // Laplacian's six neighbours.
    auto transport = [&](auto sc, const vec4<V>& q0, const vec4<V>& qm2, const vec4<V>& qm1, const vec4<V>& qp1,
                         const vec4<V>& qp2, const vec4<V>& lxp, const vec4<V>& lxm, const vec4<V>& lyp,
                         const vec4<V>& lym, const vec4<V>& lzp, const vec4<V>& lzm) {
        constexpr int s = decltype(sc)::value;
        constexpr int i0 = 2 * s - 1, i1 = 2 * s;
        constexpr int ex = EX[i0], ey = EY[i0], ez = EZ[i0];
        // +e: upwind stencil x - 2e, x - e, x, x + e; -e: x + 2e, x + e, x, x - e
        const V lap0 = (lxp.x + lxm.x) + (lyp.x + lym.x) + (lzp.x + lzm.x) - V(6) * q0.x;
        const V lap1 = (lxp.z + lxm.z) + (lyp.z + lym.z) + (lzp.z + lzm.z) - V(6) * q0.z;
        const V fv0 = q0.x - cour * ((q0.x + slope * minmod(q0.x - qm1.x, qp1.x - q0.x)) -
                                     (qm1.x + slope * minmod(qm1.x - qm2.x, q0.x - qm1.x))) + kv * lap0;
        const V fv1 = q0.z - cour * ((q0.z + slope * minmod(q0.z - qp1.z, qm1.z - q0.z)) -
                                     (qp1.z + slope * minmod(qp1.z - qp2.z, q0.z - qp1.z))) + kv * lap1;
        const V gv0 = q0.y - cour * ((q0.y + slope * minmod(q0.y - qm1.y, qp1.y - q0.y)) -
                                     (qm1.y + slope * minmod(qm1.y - qm2.y, q0.y - qm1.y)));
        const V gv1 = q0.w - cour * ((q0.w + slope * minmod(q0.w - qp1.w, qm1.w - q0.w)) -
                                     (qp1.w + slope * minmod(qp1.w - qp2.w, q0.w - qp1.w)));
        Fv[i0] = fv0;
        Fv[i1] = fv1;
        Gv[i0] = gv0;
        Gv[i1] = gv1;
        const V sum = fv0 + fv1, dif = fv0 - fv1;
        t00 += sum;
        n0 += gv0 + gv1;
        if (ex) t0x += ex * dif;
        if (ey) t0y += ey * dif;
        if (ez) t0z += ez * dif;
        if (ex) txx += sum;
        if (ey) tyy += sum;
        if (ez) tzz += sum;
        if (ex * ey) txy += (ex * ey) * sum;
        if (ex * ez) txz += (ex * ez) * sum;
        if (ey * ez) tyz += (ey * ez) * sum;
    };
    // a slot whose link runs along one axis finds its points x -+ e among the Laplacian's neighbours
    if constexpr (!dquad_layout<TS>()) {
        {
            const vec2<V> fg0 = ldv2<V>(sd, quad_index(K, 0, cell));
            Fv[0] = fg0.x;
            Gv[0] = fg0.y;
            t00 = Fv[0];
            n0 = Gv[0];
        }
        static_for<1>([&](auto ic) {
            constexpr int s = decltype(ic)::value;
            if constexpr (s <= 9) {
                constexpr int i0 = 2 * s - 1;
                constexpr int ex = EX[i0], ey = EY[i0], ez = EZ[i0];
                const TS* __restrict__ qa = sd + quad_index(K, s, 0);  // uniform base of slot s
                auto ldq = [&](int off) { return ldv4<V>(qa, 4 * (int64_t)(cell + off)); };
                const vec4<V> q0 = ldq(0), qm2 = ldq(nb.at(-2 * ex, -2 * ey, -2 * ez)), qm1 = ldq(nb.at(-ex, -ey, -ez)),
                              qp1 = ldq(nb.at(ex, ey, ez)), qp2 = ldq(nb.at(2 * ex, 2 * ey, 2 * ez));
                constexpr bool ax = (ex != 0) + (ey != 0) + (ez != 0) == 1;
                const vec4<V> lxp = ax && ex ? qp1 : ldq(lap_xp), lxm = ax && ex ? qm1 : ldq(lap_xm);
                const vec4<V> lyp = ax && ey ? qp1 : ldq(lap_yp), lym = ax && ey ? qm1 : ldq(lap_ym);
                const vec4<V> lzp = ax && ez ? qp1 : ldq(lap_zp), lzm = ax && ez ? qm1 : ldq(lap_zm);
                transport(ic, q0, qm2, qm1, qp1, qp2, lxp, lxm, lyp, lym, lzp, lzm);
                V(&F_)[Q] = Fv;
                V(&G_)[Q] = Gv;
                if constexpr (s % RMHDLB_QGROUP == 0 || s == 9)
                    asm volatile("" : "+v"(F_[i0]), "+v"(F_[i0 + 1]), "+v"(G_[i0]), "+v"(G_[i0 + 1])::"memory");
            }
        });
    } else {
        // record r: slots a = 2r + 1 and b = 2r + 2 (record 4: slot 9 and the rest pair); the centre and
        // the Laplacian's points take one 16-byte load for both slots, the link points an 8-byte one
        static_for<0>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            if constexpr (r < DQUAD_RECORDS) {
                constexpr int sa = 2 * r + 1, sb = r < 4 ? 2 * r + 2 : 0;
                const TS* __restrict__ ra = sd + dquad_index(K, r, 0);  // uniform base of record r
                auto ld8 = [&](int off, vec4<V>& lo, vec4<V>& hi) { ldv8<V>(ra, 8 * (int64_t)(cell + off), lo, hi); };
                auto ld4 = [&](int off, int half) { return ldv4<V>(ra, 8 * (int64_t)(cell + off) + 4 * half); };
                vec4<V> ca, cb;
                ld8(0, ca, cb);
                vec4<V> xpa, xpb, xma, xmb, ypa, ypb, yma, ymb, zpa, zpb, zma, zmb;
                if constexpr (sb != 0) {
                    ld8(lap_xp, xpa, xpb);
                    ld8(lap_xm, xma, xmb);
                    ld8(lap_yp, ypa, ypb);
                    ld8(lap_ym, yma, ymb);
                    ld8(lap_zp, zpa, zpb);
                    ld8(lap_zm, zma, zmb);
                } else {
                    xpa = ld4(lap_xp, 0);
                    xma = ld4(lap_xm, 0);
                    ypa = ld4(lap_yp, 0);
                    yma = ld4(lap_ym, 0);
                    zpa = ld4(lap_zp, 0);
                    zma = ld4(lap_zm, 0);
                }
                // the link points of slot s (half h of the record), reusing the Laplacian's on an axis slot
                auto links = [&](auto sc, int h, const vec4<V>& xp, const vec4<V>& xm, const vec4<V>& yp,
                                 const vec4<V>& ym, const vec4<V>& zp, const vec4<V>& zm, vec4<V>& qm2, vec4<V>& qm1,
                                 vec4<V>& qp1, vec4<V>& qp2) {
                    constexpr int s = decltype(sc)::value;
                    constexpr int ex = EX[2 * s - 1], ey = EY[2 * s - 1], ez = EZ[2 * s - 1];
                    constexpr bool ax = (ex != 0) + (ey != 0) + (ez != 0) == 1;
                    qm2 = ld4(nb.at(-2 * ex, -2 * ey, -2 * ez), h);
                    qp2 = ld4(nb.at(2 * ex, 2 * ey, 2 * ez), h);
                    if constexpr (ax && ex == 1) {
                        qp1 = xp;
                        qm1 = xm;
                    } else if constexpr (ax && ex == -1) {
                        qp1 = xm;
                        qm1 = xp;
                    } else if constexpr (ax && ey == 1) {
                        qp1 = yp;
                        qm1 = ym;
                    } else if constexpr (ax && ey == -1) {
                        qp1 = ym;
                        qm1 = yp;
                    } else if constexpr (ax && ez == 1) {
                        qp1 = zp;
                        qm1 = zm;
                    } else if constexpr (ax && ez == -1) {
                        qp1 = zm;
                        qm1 = zp;
                    } else {
                        qp1 = ld4(nb.at(ex, ey, ez), h);
                        qm1 = ld4(nb.at(-ex, -ey, -ez), h);
                    }
                };
                vec4<V> am2, am1, ap1, ap2;
                links(std::integral_constant<int, sa>{}, 0, xpa, xma, ypa, yma, zpa, zma, am2, am1, ap1, ap2);
                transport(std::integral_constant<int, sa>{}, ca, am2, am1, ap1, ap2, xpa, xma, ypa, yma, zpa, zma);
                V(&F_)[Q] = Fv;
                V(&G_)[Q] = Gv;
                asm volatile("" : "+v"(F_[2 * sa - 1]), "+v"(F_[2 * sa]), "+v"(G_[2 * sa - 1]), "+v"(G_[2 * sa])::"memory");
                if constexpr (sb != 0) {
                    vec4<V> bm2, bm1, bp1, bp2;
                    links(std::integral_constant<int, sb>{}, 1, xpb, xmb, ypb, ymb, zpb, zmb, bm2, bm1, bp1, bp2);
                    transport(std::integral_constant<int, sb>{}, cb, bm2, bm1, bp1, bp2, xpb, xmb, ypb, ymb, zpb,
                              zmb);
                    asm volatile("" : "+v"(F_[2 * sb - 1]), "+v"(F_[2 * sb]), "+v"(G_[2 * sb - 1]),
                                 "+v"(G_[2 * sb])::"memory");
                } else {  // the rest pair
                    Fv[0] = cb.x;
                    Gv[0] = cb.y;
                    t00 += Fv[0];
                    n0 += Gv[0];
                }
            }
        });
    }
    // stream h (Eq. LB_Maxwell): the pair 2m, 2m + 1 from its common source cell
    V ehx = 0, ehy = 0, ehz = 0, bx = 0, by = 0, bz = 0, hs = 0;
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const vec2<V> v = ldv2<V>(sd, hpair_index(K, m, (int64_t)cell + nb.at(-SX[k0], -SY[k0], -SZ[k0])));
        Hv[k0] = v.x;
        Hv[k0 + 1] = v.y;
        hs += v.x + v.y;
        const V d = v.x - v.y;  // population 2m + 1 has the opposite e and b
        if (EHX[k0]) ehx += EHX[k0] * d;
        if (EHY[k0]) ehy += EHY[k0] * d;
        if (EHZ[k0]) ehz += EHZ[k0] * d;
        if (BHX[k0]) bx += BHX[k0] * d;
        if (BHY[k0]) by += BHY[k0] * d;
        if (BHZ[k0]) bz += BHZ[k0] * d;
    }
    Hv[QH] = ldv<V>(sd, hrest_quad_index(K, cell));
    CellSol M;
#pragma unroll
    for (int a = 0; a < 3; ++a) M.Ep[a] = ld(se + (int64_t)a * S + cell, 0);
    {
        const TE* ex_ = se + cell;
        const TE* ey_ = se + S + cell;
        const TE* ez_ = se + 2 * S + cell;
        const double dv = ((ld(ex_, lap_xp) - ld(ex_, lap_xm)) + (ld(ey_, lap_yp) - ld(ey_, lap_ym))) +
                          (ld(ez_, lap_zp) - ld(ez_, lap_zm));
        M.rho_g = K.eps0 * K.inv_2dx * dv;
    }
    M.T00 = K.fs0 + (double)t00;
    M.N0 = K.gs0 + (double)n0;
    M.T0[0] = KAPPA * (double)t0x;
    M.T0[1] = KAPPA * (double)t0y;
    M.T0[2] = KAPPA * (double)t0z;
    M.Tab[0] = KAPPA2 * (K.fsaa + (double)txx);
    M.Tab[1] = KAPPA2 * (K.fsaa + (double)tyy);
    M.Tab[2] = KAPPA2 * (K.fsaa + (double)tzz);
    M.Tab[3] = KAPPA2 * (double)txy;
    M.Tab[4] = KAPPA2 * (double)txz;
    M.Tab[5] = KAPPA2 * (double)tyz;
    const double ec = K.c * INV_SQRT2;
    M.Epr[0] = ec * (double)ehx;
    M.Epr[1] = ec * (double)ehy;
    M.Epr[2] = ec * (double)ehz;
    M.B[0] = (double)bx;
    M.B[1] = (double)by;
    M.B[2] = (double)bz;
    // h* = 2 h_eq - h: the B part of h_eq (of the streamed B) now
    {
        const V sb0 = (V)M.B[0], sb1 = (V)M.B[1], sb2 = (V)M.B[2];
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const int k0 = 2 * m;
            const V bb = V(0.25) * (BHX[k0] * sb0 + BHY[k0] * sb1 + BHZ[k0] * sb2);
            Hv[k0] -= bb;
            Hv[k0 + 1] += bb;
        }
    }
    M.rho = (double)(Hv[QH] + hs);
    if (K.divb) apply_face_b(K, faceB, x, y, z, M.B);
    FeqCellT<V> fe;
    if constexpr ((VR & 8) != 0) {
        double Bp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Bp[a] = ld(se + (int64_t)(3 + a) * S + cell, 0);
        solve_cell<GM>(K, M, Bp, gt, &gate);
        fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, Bp, K.c, K.eps0);
    } else {
        solve_cell<GM>(K, M, M.B, gt, &gate);
        fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, M.B, K.c, K.eps0);
    }

    // collisions and stores (new deviations)
    const V rate = (V)(M.gam * K.inv_tau);
    const V wg = (V)K.wg, inv1wg = (V)(1.0 / (1.0 + K.wg));
    const V ng = (V)(M.n * M.gam);
    const V gc1 = (V)K.gc1, gc2 = (V)K.gc2, gc3b2 = (V)(K.gc3 * (M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] +
                                                              M.beta[2] * M.beta[2]));
    const V bx_ = (V)M.beta[0], by_ = (V)M.beta[1], bz_ = (V)M.beta[2];
    double fw = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if constexpr ((VR & 4) != 0) {
        bmax = fmax(bmax, sqrt(M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] + M.beta[2] * M.beta[2]));
        if (!(K.fgate > 0.0) || *K.vmax_prev < K.fgate) {
            const double cdt = K.dx * INV_SQRT2;  // c dt
            fx = cdt * K.force[cell];
            fy = cdt * K.force[K.N + cell];
            fz = cdt * K.force[2 * K.N + cell];
            fw = fx * M.beta[0] + fy * M.beta[1] + fz * M.beta[2];
        }
    }
    vec4<V> rest;  // new (f_0, g_0, 0, 0)
    {
        const V q0 = (V)K.fsh[0] - fe.template eq<0>();
        const V geq0 = (V)K.wp[0] * ng * (V(1) - gc3b2);
        V f0n = CM == 0 ? Fv[0] - rate * (Fv[0] + q0) : (Fv[0] - rate * q0) / (V(1) + rate);
        if constexpr ((VR & 4) != 0) f0n += (V)fw;
        rest.x = f0n;
        rest.y = (Gv[0] + wg * (geq0 - (V)K.gsh[0])) * inv1wg;
        rest.z = V(0);
        rest.w = V(0);
        if constexpr (!dquad_layout<TS>())
            if (active) st2<NT>(dd + quad_index(K, 0, cell), rest.x, rest.y);
    }
    put(dd + hrest_quad_index(K, cell), (V)(2.0 * M.rho) - Hv[QH]);
    // the new quad (f, g, f-bar, g-bar) of slot s
    auto collide = [&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int i0 = 2 * s - 1, i1 = 2 * s;
        constexpr int cls = i0 <= 6 ? 1 : 2;
        const V eb = EX[i0] * bx_ + EY[i0] * by_ + EZ[i0] * bz_;  // e_i0 . beta; -eb for i1
        const V q_0 = (V)K.fsh[cls] - feq_signed<i0>(fe, V(1));
        const V q_1 = (V)K.fsh[cls] - feq_signed<i0>(fe, V(-1));
        const V om0 = rate * (V(1) - V(KAPPA) * eb), om1 = rate * (V(1) + V(KAPPA) * eb);
        const V ebb = gc2 * eb * eb - gc3b2;
        const V geq_0 = (V)K.wp[cls] * ng * (V(1) + gc1 * eb + ebb);
        const V geq_1 = (V)K.wp[cls] * ng * (V(1) - gc1 * eb + ebb);
        V fn0 = CM == 0 ? Fv[i0] - om0 * (Fv[i0] + q_0) : (Fv[i0] - om0 * q_0) / (V(1) + om0);
        V fn1 = CM == 0 ? Fv[i1] - om1 * (Fv[i1] + q_1) : (Fv[i1] - om1 * q_1) / (V(1) + om1);
        if constexpr ((VR & 4) != 0) {
            constexpr double wcls = cls == 1 ? 99.0 / 722.0 : 9.0 / 361.0;  // D3Q19 weights
            const double fe_ = (19.0 / 9.0) * wcls / KAPPA * (EX[i0] * fx + EY[i0] * fy + EZ[i0] * fz);
            fn0 += (V)fe_;
            fn1 += (V)(-fe_);
        }
        vec4<V> q;
        q.x = fn0;
        q.y = (Gv[i0] + wg * (geq_0 - (V)K.gsh[cls])) * inv1wg;
        q.z = fn1;
        q.w = (Gv[i1] + wg * (geq_1 - (V)K.gsh[cls])) * inv1wg;
        return q;
    };
    if constexpr (!dquad_layout<TS>()) {
        static_for<1>([&](auto ic) {
            constexpr int s = decltype(ic)::value;
            if constexpr (s <= 9) {
                const vec4<V> q = collide(ic);
                if (active) st4<NT>(dd + quad_index(K, s, cell), q.x, q.y, q.z, q.w);
            }
        });
    } else {
        static_for<0>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            if constexpr (r < DQUAD_RECORDS) {
                const vec4<V> a = collide(std::integral_constant<int, 2 * r + 1>{});
                if constexpr (r < 4) {
                    const vec4<V> b = collide(std::integral_constant<int, 2 * r + 2>{});
                    if (active) st8<NT>(dd + dquad_index(K, r, cell), a, b);
                } else {
                    if (active) st8<NT>(dd + dquad_index(K, r, cell), a, rest);
                }
            }
        });
    }
    const V cj = (V)(1.0 / (16.0 * 1.4142135623730951 * K.c)), ce = (V)(1.0 / (8.0 * 1.4142135623730951 * K.c));
    const V J0 = (V)M.J[0], J1 = (V)M.J[1], J2 = (V)M.J[2];
    const V E0 = (V)M.E[0], E1 = (V)M.E[1], E2 = (V)M.E[2];
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const V hj = cj * (SX[k0] * J0 + SY[k0] * J1 + SZ[k0] * J2);
        const V he = ce * (EHX[k0] * E0 + EHY[k0] * E1 + EHZ[k0] * E2);
        if (active)
            st2<NT>(dd + hpair_index(K, m, cell), V(2) * (hj + he) - Hv[k0], V(2) * (hj - he) - Hv[k0 + 1]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) put(de + (int64_t)a * S + cell, M.E[a]);
    if constexpr ((VR & 8) != 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) put(de + (int64_t)(3 + a) * S + cell, M.B[a]);
    }
}

// ------------------------------------------------------------------ kernels

// One block owns a PXT x (128 / PXT) group of rows of cells (two lanes per
// cell), yw such groups stacked along y (a tile of PXT x (128 / PXT) yw
// cells), and walks zb z-planes, the yw groups of a plane one after another.  A chunk of zg * zb planes is shared by zg blocks
// per column: block r of the zg takes planes r, r + zg, r + 2 zg, ... of the
// chunk, so that the zg blocks of a column run at neighbouring planes at the
// same time and the z-neighbour planes of the stencil are fetched once into
// L2 for all of them (zg = 1: one block walks zb consecutive planes).  Blocks
// are numbered column-fastest within a chunk, the zg blocks of a column next
// to each other, and XCD k receives the contiguous block range [k P, (k + 1) P):
// the columns one XCD runs at the same time are neighbours marching through
// the same planes, so the y-halo meets in that XCD's L2 as well.
// With the learned guess the network runs on whole wavefronts, so lanes past
// a ragged edge stay and compute a copy of the edge cell without storing it.
template <bool NT, typename TS, typename TE, typename V, int GM, int PXT, int VR = 0>
__device__ __forceinline__ void fused_block(const TS* __restrict__ sd, const TE* __restrict__ se,
                                            TS* __restrict__ dd, TE* __restrict__ de,
                                            const double* __restrict__ faceB, const GuessTables* __restrict__ gt,
                                            const Consts& K, int tiles_x, int ncol, int zb, int zg, int yw, int b) {
    // pair layout (FP64): 128 cells per row group, two lanes each; quad and double-quad layouts (FP32,
    // FP16): 256 cells, one lane each
    constexpr bool ONE = quad_layout<TS>();
    constexpr int PYT = (ONE ? 256 : 128) / PXT;
    const int per = ncol * zg, zc = b / per, r = b % per;
    const int col = r / zg, zoff = r % zg;
    const int tx = col % tiles_x, ty = col / tiles_x;
    // pair layout: cell c of a row group is lane c % 32 (h = 0) and lane c % 32 + 32 (h = 1) of
    // wavefront c / 32; quad layout: cell c is thread c
    const int lane = threadIdx.x & 63;
    const int c = ONE ? (int)threadIdx.x : (int)(threadIdx.x >> 6) * 32 + (lane & 31), h = ONE ? 0 : lane >> 5;
    const int xr = tx * PXT + (c % PXT);
    int x = xr;
    const int ybase = ty * PYT * yw + c / PXT;
    // with the force every lane stays (the wavefront's largest |beta| is
    // reduced over all 64 lanes)
    constexpr bool all_lanes = GM == GUESS_PAIR || GM == GUESS_SINGLE || (VR & 4) != 0;
    // row groups of this lane that lie inside the grid (the later groups are further along y)
    int ng = yw;
    if (ybase >= K.ny) ng = 0;
    else if (ybase + (yw - 1) * PYT >= K.ny) ng = (K.ny - 1 - ybase) / PYT + 1;
    if constexpr (!all_lanes) {
        if (x >= K.nx || ng == 0) return;  // both lanes of a pair leave together
    } else {
        x = min(x, K.nx - 1);
    }
    const int z0 = zc * zb * zg, z1 = min(K.nz, z0 + zb * zg);
    double bmax = 0.0;
    bool gate = false;  // a cell of the walk lay above the guess's gate (uniform over the wavefront)
    // In FP64 and FP16 the lane's coordinates are made opaque at every plane,
    // so that the x- and y-parts of the neighbour table are recomputed per
    // plane (a few integer operations) instead of being kept across the walk:
    // in FP64, whose cell code is at the register limit, that took 7 scratch
    // reloads per plane out of the loop; in FP16 (double-quad layout) it is
    // 0.4-1.2 % faster.  FP32 keeps them (recomputing them there measured 6 %
    // slower).
    constexpr bool opaque = sizeof(TS) != 4;
    const int groups = all_lanes ? yw : ng;
    for (int z = z0 + zoff; z < z1; z += zg) {
        for (int j = 0; j < groups; ++j) {
            const int yj = ybase + j * PYT;
            const bool active = xr < K.nx && yj < K.ny;
            int xp = x, yp = all_lanes ? min(yj, K.ny - 1) : yj, hp = h;
            if constexpr (opaque) asm volatile("" : "+v"(xp), "+v"(yp), "+v"(hp));
            const int cell = xp + K.nx * (yp + K.ny * z);
            const Nbr nb = make_nbr<true>(K, xp, yp, z);
            if constexpr (ONE)
                quad_cell<NT, TS, TE, V, GM, VR>(sd, se, dd, de, faceB, gt, K, cell, nb, xp, yp, z,
                                                 all_lanes ? active : true, bmax, gate);
            else
                pair_cell<NT, TS, TE, V, GM, VR>(sd, se, dd, de, faceB, gt, K, cell, nb, hp, xp, yp, z,
                                                 all_lanes ? active : true, bmax, gate);
        }
    }
    if constexpr (GM != GUESS_NONE) open_gate(K, gate);
    if constexpr ((VR & 4) != 0) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
        if (lane == 0) K.vmax_part[(int64_t)b * (PTPB / 64) + (threadIdx.x >> 6)] = bmax;
    }
}

template <bool NT, typename TS, typename TE, typename V, int GM, int PXT, int VR>
__global__ __launch_bounds__(PTPB, (fused_waves<TS, GM>())) void k_fused_step(const TS* __restrict__ sd, const TE* __restrict__ se,
                                                        TS* __restrict__ dd, TE* __restrict__ de,
                                                        const double* __restrict__ faceB,
                                                        const GuessTables* __restrict__ gt, Consts K,
                                                        int tiles_x, int ncol, int zb, int zg, int yw, int nblk) {
    const int b = tile_of_block(nblk);
    if (b >= nblk) return;  // uniform over the block
    // With the guess enabled every step launches the network kernel and the monitor kernel (its own
    // instantiation, so that it carries none of the network's registers); the one the gate does not
    // select leaves at once (uniform over the grid).
    if constexpr (GM == GUESS_MONITOR) {
        if (*K.gflag_rd == K.gstep - 1) return;
    } else if constexpr (GM != GUESS_NONE) {
        if (*K.gflag_rd != K.gstep - 1) return;
        if (blockIdx.x == 0 && threadIdx.x == 0 && K.gcount) *K.gcount += 1;  // one writer per step
    }
    fused_block<NT, TS, TE, V, GM, PXT, VR>(sd, se, dd, de, faceB, gt, K, tiles_x, ncol, zb, zg, yw, b);
}

// Index of the instance whose range [first[i], first[i + 1]) holds v (first
// is ascending with first[0] = 0); uniform over the block.
template <typename Get>
__device__ __forceinline__ int find_instance(int ninst, int64_t v, Get first) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Batched step: the blocks of every instance in one launch.  Block b is
// mapped XCD-aware over the whole batch, then to its instance by the prefix
// table of block counts, so neighbouring tiles of one instance still share
// an XCD.  parity selects which of each instance's buffers is read.  WV:
// waves per SIMD the kernel is compiled for (the occupancy the batch tuner
// sweeps).
template <bool NT, typename TS, typename TE, typename V, int PXT, int WV>
__global__ __launch_bounds__(PTPB, WV) void k_fused_batch(const BatchInst* __restrict__ I, int ninst, int total,
                                                          int parity) {
    const int b = tile_of_block(total);
    if (b >= total) return;
    const int i = find_instance(ninst, b, [&](int j) { return I[j].blk0; });
    const BatchInst& B = I[i];
    fused_block<NT, TS, TE, V, GUESS_NONE, PXT>(
        (const TS*)B.dist[parity], (const TE*)B.efield[parity], (TS*)B.dist[1 - parity], (TE*)B.efield[1 - parity],
        B.faceB, nullptr, B.K, B.tiles_x, B.ncol, B.zb, 1, B.yw, (int)(b - B.blk0));
}

// B of Eq. Cal_B at a cell from the streamed h (population order, FP64).
template <typename TS>
__device__ __forceinline__ double streamed_B(const TS* __restrict__ src, const Consts& K, int comp, int x, int y,
                                             int z) {
    const Nbr nb = make_nbr<true>(K, x, y, z);
    const int cell = x + K.nx * (y + K.ny * z);
    double b = 0.0;
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const int bk = comp == 0 ? BHX[k] : (comp == 1 ? BHY[k] : BHZ[k]);
        if (bk) b += bk * ld(src, h_at<TS>(K, k, (int64_t)cell + nb.at(-SX[k], -SY[k], -SZ[k])));
    }
    return b;
}

// Normal B of the open-face cells for this step (Sec. IV, KH set-up): in a
// cell on an open face of axis a (not an edge or corner cell) the discrete
// divergence is made zero with
// the streamed B of the inner neighbour and the tangential derivatives of
// the streamed B:  low face  B_a = B_a(x + e_a) + dx sum_{b != a} d_b B_b,
//                  high face B_a = B_a(x - e_a) - dx sum_{b != a} d_b B_b.
// One thread per face cell over the six faces; inactive faces return.
template <typename TS>
__device__ __forceinline__ void face_b_cell(const TS* __restrict__ src, const Consts& K, double* __restrict__ faceB,
                                            int64_t i) {
    if (i >= K.fo[6]) return;
    int f = 0;
    while (f < 5 && i >= K.fo[f + 1]) ++f;
    const int a = f >> 1, high = f & 1;
    if (!(high ? K.open_hi[a] : K.open_lo[a])) return;
    const int64_t j = i - K.fo[f];
    int x, y, z;
    if (a == 0) {
        y = (int)(j % K.ny);
        z = (int)(j / K.ny);
        x = high ? K.nx - 1 : 0;
    } else if (a == 1) {
        x = (int)(j % K.nx);
        z = (int)(j / K.nx);
        y = high ? K.ny - 1 : 0;
    } else {
        x = (int)(j % K.nx);
        y = (int)(j / K.nx);
        z = high ? K.nz - 1 : 0;
    }
    if (on_other_face(K, a, x, y, z)) return;  // edge and corner cells keep the streamed B
    double dsum = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (b != a)
            dsum += axis_derivative(K, b, x, y, z, [&](int xx, int yy, int zz) { return streamed_B(src, K, b, xx, yy, zz); });
    const int s = high ? -1 : 1;
    const double inner = streamed_B(src, K, a, x + s * (a == 0), y + s * (a == 1), z + s * (a == 2));
    faceB[i] = high ? inner - K.dx * dsum : inner + K.dx * dsum;
}

template <typename TS>
__global__ __launch_bounds__(256) void k_face_b(const TS* __restrict__ src, Consts K, double* __restrict__ faceB) {
    face_b_cell(src, K, faceB, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// The face pass of every instance of a batch in one launch.
template <typename TS>
__global__ __launch_bounds__(256) void k_face_b_batch(const BatchInst* __restrict__ I, int ninst, int64_t total,
                                                      int parity) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= total) return;
    const int i = find_instance(ninst, g, [&](int j) { return I[j].face0; });
    const BatchInst& B = I[i];
    if (!B.K.divb) return;
    face_b_cell((const TS*)B.dist[parity], B.K, B.faceB, g - B.face0);
}

// Persistent batched run: nsteps steps in one cooperative launch whose grid
// (a multiple of 8) is no larger than the blocks resident at once.  The tiles
// of a step are dealt as k_fused_batch deals its blocks: XCD x (blocks g with
// g % 8 == x, as the hardware deals blocks to XCDs) runs the contiguous tile
// range [x P, (x + 1) P), and its blocks take the next tile of that range
// from a counter, in order and as they become free (each block takes its
// next one while its current one runs), so that the tiles in flight
// together stay neighbours.  next holds two sets of 8 counters, zero
// at launch: step k counts in set k % 2, and the first block of each group
// clears its counter of the other set (last used in step k - 1, whose fetches
// all ended before the barrier).  All blocks meet at a grid barrier after
// each step (the next one reads what it wrote).  No face pass: batches with
// the open-face adjustment are stepped by graph replays.  Every block reaches
// every barrier: no thread leaves the kernel early, and a fetch loop ends
// once its counter passes P.
template <bool NT, typename TS, typename TE, typename V, int PXT, int WV>
__global__ __launch_bounds__(PTPB, WV) void k_fused_batch_persistent(const BatchInst* __restrict__ I, int ninst,
                                                                     int total, int parity0, int nsteps,
                                                                     int* __restrict__ next) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ int tile_sh;
    const int P = (total + 7) / 8;
    const int x = blockIdx.x % 8;
    for (int k = 0; k < nsteps; ++k) {
        const int parity = (parity0 + k) & 1;
        int* cnt = next + (k & 1) * 8 + x;
        if (blockIdx.x < 8 && threadIdx.x == 0) atomicExch(next + ((k + 1) & 1) * 8 + x, 0);
        // the next tile is taken while the current one runs, so the counter's round trip is hidden
        if (threadIdx.x == 0) tile_sh = atomicAdd(cnt, 1);
        __syncthreads();
        int j = tile_sh;
        __syncthreads();
        while (j < P) {  // j is uniform over the block
            int nj = 0;
            if (threadIdx.x == 0) nj = atomicAdd(cnt, 1);
            const int b = x * P + j;
            if (b < total) {
                const int i = find_instance(ninst, b, [&](int jj) { return I[jj].blk0; });
                const BatchInst& B = I[i];
                fused_block<NT, TS, TE, V, GUESS_NONE, PXT>(
                    (const TS*)B.dist[parity], (const TE*)B.efield[parity], (TS*)B.dist[1 - parity],
                    (TE*)B.efield[1 - parity], B.faceB, nullptr, B.K, B.tiles_x, B.ncol, B.zb, 1, B.yw,
                    (int)(b - B.blk0));
            }
            if (threadIdx.x == 0) tile_sh = nj;
            __syncthreads();
            j = tile_sh;
            __syncthreads();
        }
        grid.sync();
    }
}

// Deterministic (key, index) minimum, ties to the lower index; NaN keys never win.
__device__ __forceinline__ void argmin_merge(double& k, double& i, double k2, double i2) {
    if (k2 < k || (k2 == k && i2 < i)) {
        k = k2;
        i = i2;
    }
}

__device__ __forceinline__ void block_argmin(double k, double i, double* __restrict__ out) {
    __shared__ double shk[RED_WAVES], shi[RED_WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) argmin_merge(k, i, __shfl_xor(k, o, 64), __shfl_xor(i, o, 64));
    if (lane == 0) {
        shk[wave] = k;
        shi[wave] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bk = shk[0], bi = shi[0];
        for (int w = 1; w < RED_WAVES; ++w) argmin_merge(bk, bi, shk[w], shi[w]);
        out[0] = bk;
        out[1] = bi;
    }
}

constexpr double NO_INDEX = 9.0e15;  // larger than any cell index, exact in FP64

// Primitives of the current state and per-block partial diagnostics:
// part[blk * NPART + j], j = T00, N0, T0x, T0y, T0z, em energy, rho, iters,
// failed, then 16 Newton-iteration bins, then learned-guess fallbacks;
// null-search partials (least B_x^2 + B_y^2 in the band and its cell) in
// nullp[2 blk ..]; B and E^z of every cell into scratch (4 arrays of N).
// Every thread runs the cell pass (on the edge cell when past a ragged edge,
// so that the network sees whole wavefronts); only real cells write.
template <typename TS, typename TE, int GM>
__global__ __launch_bounds__(TPB) void k_moments(const TS* __restrict__ src, const TE* __restrict__ esrc,
                                                 const double* __restrict__ faceB,
                                                 const GuessTables* __restrict__ gt, Consts K, int tiles_x,
                                                 int tiles_y, int ntiles, OutPtrs out, double* __restrict__ scratch,
                                                 double* __restrict__ part, double* __restrict__ nullp) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;  // uniform over the block
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x0 = tx * TX + (threadIdx.x % TX), y0 = ty * TY + (threadIdx.x / TX);
    const bool active = x0 < K.nx && y0 < K.ny;
    const int x = min(x0, K.nx - 1), y = min(y0, K.ny - 1);
    double v[NPART] = {0};
    double key = __builtin_inf(), idx = NO_INDEX;
    const int cell = x + K.nx * (y + K.ny * z);
    const Nbr nb = make_nbr<true>(K, x, y, z);
    Macro M;
    if constexpr (GM == GUESS_NONE)
        macroscopic<GM>(src, esrc, faceB, gt, K, cell, nb, x, y, z, M);
    else if (*K.gflag_rd == K.gstep - 1)  // the guess the next step would take
        macroscopic<GM>(src, esrc, faceB, gt, K, cell, nb, x, y, z, M);
    else
        macroscopic<GUESS_MONITOR>(src, esrc, faceB, gt, K, cell, nb, x, y, z, M);
    if (active) {
        const double c = K.c;
        if (out.n) out.n[cell] = M.n;
        if (out.p) out.p[cell] = M.p;
        if (out.eps) out.eps[cell] = M.eps;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (out.u[a]) out.u[a][cell] = c * M.beta[a];
            if (out.E[a]) out.E[a][cell] = M.E[a];
            if (out.B[a]) out.B[a][cell] = M.B[a];
            if (out.J[a]) out.J[a][cell] = M.J[a];
            scratch[(int64_t)a * K.N + cell] = M.B[a];
        }
        scratch[3 * K.N + cell] = M.E[2];
        if (out.rho_c) out.rho_c[cell] = M.rho;
        v[0] = M.T00;
        v[1] = M.N0;
        v[2] = M.T0[0];
        v[3] = M.T0[1];
        v[4] = M.T0[2];
        const double E2 = M.E[0] * M.E[0] + M.E[1] * M.E[1] + M.E[2] * M.E[2];
        const double B2 = M.B[0] * M.B[0] + M.B[1] * M.B[1] + M.B[2] * M.B[2];
        v[5] = 0.5 * K.eps0 * (E2 + c * c * B2);
        v[6] = M.rho;
        v[7] = M.iters;
        v[8] = M.ok ? 0.0 : 1.0;
        const int bin = M.iters < 15 ? (M.iters > 0 ? M.iters : 0) : 15;
#pragma unroll
        for (int k = 0; k < 16; ++k) v[9 + k] = bin == k ? 1.0 : 0.0;
        v[25] = M.fallback;
        // |y_j| <= band with cell centres y_j = j + 1/2 - ny/2
        const int dy = 2 * y + 1 - K.ny;
        if ((dy < 0 ? -dy : dy) <= 2 * K.band) {
            const double kb = fma(M.B[0], M.B[0], M.B[1] * M.B[1]);
            if (kb == kb) {
                key = kb;
                idx = (double)cell;
            }
        }
    }
    block_sum<NPART>(v, part + (int64_t)tile * NPART);
    block_argmin(key, idx, nullp + 2 * (int64_t)tile);
}

// max |div B| per block from the B written by k_moments (the derivative
// operator of the normal-B adjustment).
__global__ __launch_bounds__(TPB) void k_divb(const double* __restrict__ Bs, Consts K, int tiles_x, int tiles_y,
                                              int ntiles, double* __restrict__ part) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    double v[1] = {0.0};
    if (x < K.nx && y < K.ny) {
        double dv = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double* Ba = Bs + (int64_t)a * K.N;
            dv += axis_derivative(K, a, x, y, z, [&](int xx, int yy, int zz) { return Ba[xx + K.nx * (yy + K.ny * zz)]; });
        }
        v[0] = fabs(dv);
    }
    block_max1(v[0], part + tile);
}

// Null point over the per-block partials, then R = (E^z - E^z_0) / B0 there.
// out[0] = R, out[1] = null cell (-1: none), out[2] = B0.
__global__ __launch_bounds__(TPB) void k_null_reduce(const double* __restrict__ nullp, int nblk,
                                                     const double* __restrict__ ez, const double* __restrict__ ez0,
                                                     const double* __restrict__ b0, double* __restrict__ out) {
    __shared__ double res[2];
    double k = __builtin_inf(), i = NO_INDEX;
    for (int b = threadIdx.x; b < nblk; b += TPB) argmin_merge(k, i, nullp[2 * (int64_t)b], nullp[2 * (int64_t)b + 1]);
    block_argmin(k, i, res);
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool found = res[1] < NO_INDEX;
        const int64_t c = found ? (int64_t)res[1] : -1;
        out[0] = found ? (ez[c] - ez0[c]) / b0[0] : __builtin_nan("");
        out[1] = (double)c;
        out[2] = b0[0];
    }
}

// Fixed-order reduction of the per-block partials by one block.
// Largest |beta| of a forced step from its per-wavefront partials (which are
// cleared for the next step); one block.
__global__ __launch_bounds__(TPB) void k_vmax_reduce(double* __restrict__ part, int64_t n, double* __restrict__ out) {
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += TPB) {
        m = fmax(m, part[i]);
        part[i] = 0.0;
    }
    __shared__ double sh[TPB / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int w = 1; w < TPB / 64; ++w) r = fmax(r, sh[w]);
        *out = r;
    }
}

__global__ __launch_bounds__(TPB) void k_reduce(const double* __restrict__ part, int nblk, int width, int is_max,
                                                double* __restrict__ out) {
    for (int j = 0; j < width; ++j) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += TPB) {
            const double v = part[(int64_t)b * width + j];
            acc = is_max ? fmax(acc, v) : acc + v;
        }
        double r = is_max ? block_max_value(acc) : block_sum_value(acc);
        if (threadIdx.x == 0) out[j] = r;
        __syncthreads();
    }
}

// Sums of eps = n c^2 + p / (Gamma - 1) and n over the initial fields (the
// references of the stored deviations).
__global__ __launch_bounds__(TPB) void k_init_ref(InPtrs in, Consts K, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < K.N) {
        v[0] = in.n[i] * K.c * K.c + in.p[i] / K.gm1;
        v[1] = in.n[i];
    }
    block_sum<2>(v, part + (int64_t)blockIdx.x * 2);
}

// Largest B^2 of the initial fields (as fma(B_x, B_x, fma(B_y, B_y, B_z B_z))), per block.
__global__ __launch_bounds__(TPB) void k_init_bmax(InPtrs in, Consts K, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    double v = 0.0;
    if (i < K.N) v = fma(in.B[0][i], in.B[0][i], fma(in.B[1][i], in.B[1][i], in.B[2][i] * in.B[2][i]));
    block_max1(v, part + blockIdx.x);
}

__global__ void k_sqrt1(double* __restrict__ v) {
    if (threadIdx.x == 0) v[0] = sqrt(v[0]);
}

// Face cells with |u| >= c, n <= 0 or p < 0, per block.
__global__ __launch_bounds__(TPB) void k_face_check(FacePtrs in, Consts K, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    double bad[1] = {0.0};
    if (i < (int64_t)K.nx * K.ny) {
        const double u2 = in.u[0][i] * in.u[0][i] + in.u[1][i] * in.u[1][i] + in.u[2][i] * in.u[2][i];
        bad[0] = (u2 < K.c * K.c && in.n[i] > 0.0 && in.p[i] >= 0.0) ? 0.0 : 1.0;
    }
    block_sum<1>(bad, part + blockIdx.x);
}

// Ghost planes of a driven low-z face: the post-collision state of a fully
// relaxed cell with the prescribed fields -- f_eq and g_eq of (n, p, u,
// E = -u x B, B) (stored minus their shifts), h* = h_eq of (J, E + q J, B)
// with J of Eq. Ohm at zero charge (h* = h_eq is the fixed point of the
// tau_h = 1/2 collision), rest h* = 0 and E_prev = E; both planes the same.
// dd, de point at cell 0 of the state buffer; the planes sit just below it.
template <typename TS, typename TE>
__global__ __launch_bounds__(TPB) void k_init_ghost(FacePtrs in, Consts K, TS* __restrict__ dd, TE* __restrict__ de) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t plane = (int64_t)K.nx * K.ny;
    if (i >= plane) return;
    const double c = K.c, c2 = c * c;
    double u[3], Bv[3], beta[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = in.u[a][i];
        Bv[a] = in.B[a][i];
        beta[a] = u[a] / c;
    }
    const double E[3] = {-(u[1] * Bv[2] - u[2] * Bv[1]), -(u[2] * Bv[0] - u[0] * Bv[2]), -(u[0] * Bv[1] - u[1] * Bv[0])};
    const double n = in.n[i], p = in.p[i];
    const double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    const double gam = 1.0 / sqrt(1.0 - b2);
    const double eps = n * c2 + p / K.gm1;
    const double uxB[3] = {u[1] * Bv[2] - u[2] * Bv[1], u[2] * Bv[0] - u[0] * Bv[2], u[0] * Bv[1] - u[1] * Bv[0]};
    const double Eu = (E[0] * u[0] + E[1] * u[1] + E[2] * u[2]) / c2;
    double J[3], Epr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        J[a] = K.sigma * gam * (E[a] + uxB[a] - Eu * u[a]);
        Epr[a] = E[a] + K.q * J[a];
    }
    FeqCell fe;
    fe.setup(eps, p, gam, beta, E, Bv, c, K.eps0);
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * c), ce = 1.0 / (8.0 * 1.4142135623730951 * c);
    for (int layer = 1; layer <= 2; ++layer) {
        const int64_t g = i - layer * plane;  // offset of the ghost cell from cell 0
        static_for<0>([&](auto ic) {
            constexpr int q = decltype(ic)::value;
            const double eb = EX[q] * beta[0] + EY[q] * beta[1] + EZ[q] * beta[2];
            const double wpi = q == 0 ? K.wp[0] : (q <= 6 ? K.wp[1] : K.wp[2]);
            dd[f_at<TS>(K, q, g)] = static_cast<TS>(fe.template eq<q>() - fshift(K, q));
            dd[g_at<TS>(K, q, g)] =
                static_cast<TS>(wpi * n * gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * b2) - gshift(K, q));
        });
#pragma unroll
        for (int k = 0; k < QH; ++k) {
            const double heq = cj * (SX[k] * J[0] + SY[k] * J[1] + SZ[k] * J[2]) +
                               ce * (EHX[k] * Epr[0] + EHY[k] * Epr[1] + EHZ[k] * Epr[2]) +
                               0.125 * (BHX[k] * Bv[0] + BHY[k] * Bv[1] + BHZ[k] * Bv[2]);
            dd[h_at<TS>(K, k, g)] = static_cast<TS>(heq);
        }
        dd[h_at<TS>(K, QH, g)] = static_cast<TS>(0.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) de[(int64_t)a * K.stride + g] = static_cast<TE>(E[a]);
        if (K.bprev)
#pragma unroll
            for (int a = 0; a < 3; ++a) de[(int64_t)(3 + a) * K.stride + g] = static_cast<TE>(Bv[a]);
    }
}

// Initial state, pass 1: J0 from Eq. Ohm with the Gauss charge of E0, and
// E'0 = E0 + (dt/2) mu0 c^2 J0 (Reading of the initial h), into scratch.
__global__ __launch_bounds__(TPB) void k_init_current(InPtrs in, Consts K, int tiles_x, int tiles_y, int ntiles,
                                                      double* __restrict__ scr) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    if (x >= K.nx || y >= K.ny) return;
    const int cell = x + K.nx * (y + K.ny * z);
    const Nbr nb = make_nbr<false>(K, x, y, z);
    const double c = K.c, c2 = c * c;
    double u[3], E[3], B[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = in.u[a][cell];
        E[a] = in.E[a][cell];
        B[a] = in.B[a][cell];
    }
    const double rg = K.eps0 * K.inv_2dx *
                      ((in.E[0][cell + nb.at(1, 0, 0)] - in.E[0][cell + nb.at(-1, 0, 0)]) +
                       (in.E[1][cell + nb.at(0, 1, 0)] - in.E[1][cell + nb.at(0, -1, 0)]) +
                       (in.E[2][cell + nb.at(0, 0, 1)] - in.E[2][cell + nb.at(0, 0, -1)]));
    const double gam = 1.0 / sqrt(1.0 - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / c2);
    const double uxB[3] = {u[1] * B[2] - u[2] * B[1], u[2] * B[0] - u[0] * B[2], u[0] * B[1] - u[1] * B[0]};
    const double Eu = (E[0] * u[0] + E[1] * u[1] + E[2] * u[2]) / c2;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double J = K.sigma * gam * (E[a] + uxB[a] - Eu * u[a]) + rg * u[a];
        scr[(int64_t)a * K.N + cell] = J;
        scr[(int64_t)(3 + a) * K.N + cell] = E[a] + K.q * J;
    }
}

// Initial state, pass 2: f* = f_eq, g* = g_eq (stored minus their shifts),
// h*_k(x) = h_eq-form at x + s_k, h*_rest = rho_c, E_prev = E0.
template <typename TS, typename TE>
__global__ __launch_bounds__(TPB) void k_init_state(InPtrs in, Consts K, int tiles_x, int tiles_y, int ntiles,
                                                    const double* __restrict__ scr, TS* __restrict__ dst,
                                                    TE* __restrict__ edst) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    if (x >= K.nx || y >= K.ny) return;
    const int cell = x + K.nx * (y + K.ny * z);
    const Nbr nb = make_nbr<false>(K, x, y, z);
    const double c = K.c, c2 = c * c;
    double u[3], Ep[3], Bv[3], beta[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = in.u[a][cell];
        Ep[a] = in.E[a][cell];
        Bv[a] = in.B[a][cell];
        beta[a] = u[a] / c;
    }
    const double n = in.n[cell], p = in.p[cell];
    const double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    const double gam = 1.0 / sqrt(1.0 - b2);
    const double eps = n * c2 + p / K.gm1;
    FeqCell fe;
    fe.setup(eps, p, gam, beta, Ep, Bv, c, K.eps0);
    static_for<0>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double eb = EX[i] * beta[0] + EY[i] * beta[1] + EZ[i] * beta[2];
        const double wpi = i == 0 ? K.wp[0] : (i <= 6 ? K.wp[1] : K.wp[2]);
        dst[f_at<TS>(K, i, cell)] = static_cast<TS>(fe.template eq<i>() - fshift(K, i));
        dst[g_at<TS>(K, i, cell)] =
            static_cast<TS>(wpi * n * gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * b2) - gshift(K, i));
    });
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * c), ce = 1.0 / (8.0 * 1.4142135623730951 * c);
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const int t = cell + nb.at(SX[k], SY[k], SZ[k]);
        const double J0 = scr[t], J1 = scr[K.N + t], J2 = scr[2 * K.N + t];
        const double P0 = scr[3 * K.N + t], P1 = scr[4 * K.N + t], P2 = scr[5 * K.N + t];
        const double heq = cj * (SX[k] * J0 + SY[k] * J1 + SZ[k] * J2) + ce * (EHX[k] * P0 + EHY[k] * P1 + EHZ[k] * P2) +
                           0.125 * (BHX[k] * in.B[0][t] + BHY[k] * in.B[1][t] + BHZ[k] * in.B[2][t]);
        dst[h_at<TS>(K, k, cell)] = static_cast<TS>(heq);
    }
    double rho;
    if (in.rho_c) {
        rho = in.rho_c[cell];
    } else {
        rho = K.eps0 * K.inv_2dx *
              ((in.E[0][cell + nb.at(1, 0, 0)] - in.E[0][cell + nb.at(-1, 0, 0)]) +
               (in.E[1][cell + nb.at(0, 1, 0)] - in.E[1][cell + nb.at(0, -1, 0)]) +
               (in.E[2][cell + nb.at(0, 0, 1)] - in.E[2][cell + nb.at(0, 0, -1)]));
    }
    dst[h_at<TS>(K, QH, cell)] = static_cast<TS>(rho);
#pragma unroll
    for (int a = 0; a < 3; ++a) edst[(int64_t)a * K.stride + cell] = static_cast<TE>(Ep[a]);
    if (K.bprev)
#pragma unroll
        for (int a = 0; a < 3; ++a) edst[(int64_t)(3 + a) * K.stride + cell] = static_cast<TE>(Bv[a]);
}

// Raw state conversion to / from the FP64 interface layout (shifts added back).
template <typename TS, typename TE>
__global__ void k_export(const TS* __restrict__ s, const TE* __restrict__ se, double* __restrict__ d, Consts K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K.N * state_arrays(K)) return;
    const int64_t a = i / K.N, cell = i - a * K.N;
    if (a < OFF_E) {
        double v;
        if (a < OFF_G)
            v = static_cast<double>(s[f_at<TS>(K, (int)a, cell)]) + fshift(K, (int)a);
        else if (a < OFF_H)
            v = static_cast<double>(s[g_at<TS>(K, (int)(a - OFF_G), cell)]) + gshift(K, (int)(a - OFF_G));
        else
            v = static_cast<double>(s[h_at<TS>(K, (int)(a - OFF_H), cell)]);
        d[i] = v;
    } else {
        d[i] = static_cast<double>(se[(a - OFF_E) * K.stride + cell]);
    }
}

template <typename TS, typename TE>
__global__ void k_import(const double* __restrict__ s, TS* __restrict__ d, TE* __restrict__ de, Consts K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K.N * state_arrays(K)) return;
    const int64_t a = i / K.N, cell = i - a * K.N;
    if (a < OFF_E) {
        if (a < OFF_G)
            d[f_at<TS>(K, (int)a, cell)] = static_cast<TS>(s[i] - fshift(K, (int)a));
        else if (a < OFF_H)
            d[g_at<TS>(K, (int)(a - OFF_G), cell)] = static_cast<TS>(s[i] - gshift(K, (int)(a - OFF_G)));
        else
            d[h_at<TS>(K, (int)(a - OFF_H), cell)] = static_cast<TS>(s[i]);
    } else {
        de[(a - OFF_E) * K.stride + cell] = static_cast<TE>(s[i]);
    }
}

// (features, targets) of sampled cells of the current state with the plain
// recovery: cell floor(i N / ns) for sample i.  F: ns x 6, T: ns x 2 (FP64).
// Per-block partial sums of F, F^2, T, T^2 and failed cells into part (17 per block).

template <typename TS, typename TE>
__global__ __launch_bounds__(256) void k_guess_samples(const TS* __restrict__ src, const TE* __restrict__ esrc,
                                                       const double* __restrict__ faceB, Consts K, int ns,
                                                       double* __restrict__ F, double* __restrict__ T,
                                                       double* __restrict__ part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double acc[SAMPLE_SUMS] = {0};
    if (i < ns) {
        const int64_t cell = (int64_t)i * K.N / ns;
        const int x = (int)(cell % K.nx), y = (int)((cell / K.nx) % K.ny), z = (int)(cell / ((int64_t)K.nx * K.ny));
        const Nbr nb = make_nbr<true>(K, x, y, z);
        Macro M;
        macroscopic<GUESS_NONE>(src, esrc, faceB, nullptr, K, (int)cell, nb, x, y, z, M);
        double Ef, S[3], Pi[6];
        fluid_tensor(K, M, M.B, Ef, S, Pi);  // the guess is not offered with the previous-B reading
        double f[6], sn;
        f[0] = flow_ratio(Ef, S, sn);
        mlp_features(Ef, S, Pi, M.N0, sn, f);
        const double t0 = M.eps / Ef;
        const double t1 = sqrt(M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] + M.beta[2] * M.beta[2]);
        if (M.ok) {
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                F[(int64_t)i * 6 + j] = f[j];
                acc[j] = f[j];
                acc[6 + j] = f[j] * f[j];
            }
            T[(int64_t)i * 2] = t0;
            T[(int64_t)i * 2 + 1] = t1;
            acc[12] = t0;
            acc[13] = t1;
            acc[14] = t0 * t0;
            acc[15] = t1 * t1;
        } else {
            acc[16] = 1.0;
        }
    }
    block_sum<SAMPLE_SUMS>(acc, part + (int64_t)blockIdx.x * SAMPLE_SUMS);
}

// Plain copy of n 16-byte words, four per lane in flight, with the non-temporal
// hints of the step's streamed loads and stores (the reference rate of HBM).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * (256 * 4) + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
}

// ------------------------------------------------------------ host launchers

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s) {
    const int64_t blocks = (n16 + 1023) / 1024;
    if (blocks > 0)
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n16);
    return hipGetLastError();
}

static inline void grid_of(const Consts& K, int& tiles_x, int& tiles_y, int& ntiles, int& nblocks) {
    tiles_x = (K.nx + TX - 1) / TX;
    tiles_y = (K.ny + TY - 1) / TY;
    ntiles = tiles_x * tiles_y * K.nz;
    nblocks = ((ntiles + 7) / 8) * 8;
}

int num_tiles(const Consts& K) {
    int a, b, n, nb;
    grid_of(K, a, b, n, nb);
    return n;
}

template <typename TS>
hipError_t launch_face_b(const StateBuf& src, const Consts& K, double* faceB, hipStream_t s) {
    if (!K.divb) return hipSuccess;
    const int64_t blocks = (K.fo[6] + 255) / 256;
    hipLaunchKernelGGL((k_face_b<TS>), dim3((unsigned)blocks), dim3(256), 0, s, (const TS*)src.dist, K, faceB);
    return hipGetLastError();
}

void step_geometry(const Consts& K, int px, int zb, int zg, int yw, int cpb, int& tiles_x, int& ncol, int& nblk) {
    const int py = cpb / px * yw;
    tiles_x = (K.nx + px - 1) / px;
    ncol = tiles_x * ((K.ny + py - 1) / py);
    nblk = ncol * zg * ((K.nz + zg * zb - 1) / (zg * zb));
}

template <typename TS, int GM, int PXT, int VR = 0>
static void launch_fused(const TS* sd, const void* se, TS* dd, void* de, double* faceB, const GuessTables* gt,
                         const Consts& K, int zb, int zg, int yw, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    using V = typename StoreTypes<TS>::V;
    int tx, ncol, nblk;
    step_geometry(K, PXT, zb, zg, yw, cells_per_block(quad_layout<TS>()), tx, ncol, nblk);
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_fused_step<true, TS, TE, V, GM, PXT, VR>), dim3(grid), dim3(PTPB), 0, s, sd, (const TE*)se, dd,
                       (TE*)de, (const double*)faceB, gt, K, tx, ncol, zb, zg, yw, nblk);
}

template <typename TS>
hipError_t launch_step(const StateBuf& src, const StateBuf& dst, const Consts& K, const StepTuning& tune,
                       double* faceB, const GuessTables* gt, hipStream_t s) {
    hipError_t e = launch_face_b<TS>(src, K, faceB, s);
    if (e != hipSuccess) return e;
    const int zb = tune.zb > 0 ? (tune.zb < K.nz ? tune.zb : K.nz) : 1;
    // interleaved walks: zg blocks per column and chunk (the force path keeps
    // zg = 1, the geometry its per-wavefront maxima are sized for)
    const int zg = (tune.zg > 1 && !K.forced) ? tune.zg : 1;
    const TS* sd = (const TS*)src.dist;
    TS* dd = (TS*)dst.dist;
    const int vr = (K.coll ? 1 : 0) | (K.flux ? 2 : 0);
    const int yw = tune.yw > 1 && !K.forced ? tune.yw : 1;  // the force's partial maxima are sized for yw = 1
    const void* se = src.efield;
    void* de = dst.efield;
    if (K.bprev) {  // the previous-B reading: 64-wide tiles, default collision and faces, no guess or force
        if (gt || vr || K.forced) return hipErrorNotSupported;
        launch_fused<TS, GUESS_NONE, 64, 8>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    } else if (K.forced) {  // the external force: 64-wide tiles, MUSCL faces, no guess
        if (gt || K.flux) return hipErrorNotSupported;
        if (K.coll)
            launch_fused<TS, GUESS_NONE, 64, 5>(sd, se, dd, de, faceB, gt, K, zb, 1, 1, s);
        else
            launch_fused<TS, GUESS_NONE, 64, 4>(sd, se, dd, de, faceB, gt, K, zb, 1, 1, s);
        int tx, ncol, nblk;
        step_geometry(K, 64, zb, 1, 1, cells_per_block(quad_layout<TS>()), tx, ncol, nblk);
        hipLaunchKernelGGL(k_vmax_reduce, dim3(1), dim3(TPB), 0, s, K.vmax_part, (int64_t)nblk * (PTPB / 64),
                           const_cast<double*>(K.vmax_prev));
    } else if (vr) {  // the alternative readings: 64-wide tiles, no guess
        if (gt) return hipErrorNotSupported;
        if (vr == 1)
            launch_fused<TS, GUESS_NONE, 64, 1>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
        else if (vr == 2)
            launch_fused<TS, GUESS_NONE, 64, 2>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
        else
            launch_fused<TS, GUESS_NONE, 64, 3>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    } else if (gt) {  // the guess path is built for 64-wide tiles only; one cell per lane in the quad layout
        if constexpr (quad_layout<TS>())
            launch_fused<TS, GUESS_SINGLE, 64>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
        else
            launch_fused<TS, GUESS_PAIR, 64>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
        launch_fused<TS, GUESS_MONITOR, 64>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    }
    else if (tune.px == 32)
        launch_fused<TS, GUESS_NONE, 32>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    else if (tune.px == 16)
        launch_fused<TS, GUESS_NONE, 16>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    else
        launch_fused<TS, GUESS_NONE, 64>(sd, se, dd, de, faceB, gt, K, zb, zg, yw, s);
    return hipGetLastError();
}

template <typename TS, int PXT, int WV>
static void launch_batch_fused(const BatchInst* dev, int ninst, int total_blocks, int parity, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    using V = typename StoreTypes<TS>::V;
    const int grid = ((total_blocks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_fused_batch<true, TS, TE, V, PXT, WV>), dim3(grid), dim3(PTPB), 0, s, dev, ninst,
                       total_blocks, parity);
}

template <typename TS, int WV>
static void launch_batch_px(const BatchInst* dev, int ninst, int total_blocks, int px, int parity, hipStream_t s) {
    if (px == 128)
        launch_batch_fused<TS, 128, WV>(dev, ninst, total_blocks, parity, s);
    else if (px == 32)
        launch_batch_fused<TS, 32, WV>(dev, ninst, total_blocks, parity, s);
    else if (px == 16)
        launch_batch_fused<TS, 16, WV>(dev, ninst, total_blocks, parity, s);
    else
        launch_batch_fused<TS, 64, WV>(dev, ninst, total_blocks, parity, s);
}

template <typename TS>
hipError_t launch_batch(const BatchInst* dev, int ninst, int total_blocks, int64_t total_face, int px, int waves,
                        int parity, hipStream_t s) {
    if (total_face > 0)
        hipLaunchKernelGGL((k_face_b_batch<TS>), dim3((unsigned)((total_face + 255) / 256)), dim3(256), 0, s, dev,
                           ninst, total_face, parity);
    // FP32 storage (the sweep's) is built for two and three waves per SIMD;
    // FP64 and FP16 for their single-instance counts
    if constexpr (sizeof(TS) == 4) {
        if (waves == 3)
            launch_batch_px<TS, 3>(dev, ninst, total_blocks, px, parity, s);
        else
            launch_batch_px<TS, 2>(dev, ninst, total_blocks, px, parity, s);
    } else {
        launch_batch_px<TS, fused_waves<TS, 0>()>(dev, ninst, total_blocks, px, parity, s);
    }
    return hipGetLastError();
}

// Clears the persistent run's 16 tile counters (a kernel, not a memset node,
// should a caller capture the step).
__global__ void k_zero16(int* __restrict__ p) {
    if (threadIdx.x < 16) p[threadIdx.x] = 0;
}

// The persistent run's grid: the blocks resident at once (occupancy of this
// instantiation times the compute units), rounded down to a multiple of 8 and
// at most the rounded tile range.  The cooperative launch refuses a grid that
// cannot be resident as a whole, so the grid barriers always complete.
template <typename TS, int PXT, int WV>
static hipError_t launch_persistent_fused(const BatchInst* dev, int ninst, int total_blocks, int parity,
                                          int nsteps, int* next, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    using V = typename StoreTypes<TS>::V;
    const void* kern = reinterpret_cast<const void*>(&k_fused_batch_persistent<true, TS, TE, V, PXT, WV>);
    int dev_id = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev_id);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, PTPB, 0);
    if (e != hipSuccess) return e;
    const int range = (total_blocks + 7) / 8 * 8;
    const int resident = per_cu * cus / 8 * 8;
    const int grid = resident < range ? resident : range;
    if (grid < 8) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_zero16, dim3(1), dim3(64), 0, s, next);
    void* args[] = {(void*)&dev, (void*)&ninst, (void*)&total_blocks, (void*)&parity, (void*)&nsteps,
                    (void*)&next};
    return hipLaunchCooperativeKernel(kern, dim3(grid), dim3(PTPB), args, 0, s);
}

template <typename TS, int WV>
static hipError_t launch_persistent_px(const BatchInst* dev, int ninst, int total_blocks, int px, int parity,
                                       int nsteps, int* next, hipStream_t s) {
    if (px == 128)
        return launch_persistent_fused<TS, 128, WV>(dev, ninst, total_blocks, parity, nsteps, next, s);
    if (px == 32)
        return launch_persistent_fused<TS, 32, WV>(dev, ninst, total_blocks, parity, nsteps, next, s);
    if (px == 16)
        return launch_persistent_fused<TS, 16, WV>(dev, ninst, total_blocks, parity, nsteps, next, s);
    return launch_persistent_fused<TS, 64, WV>(dev, ninst, total_blocks, parity, nsteps, next, s);
}

template <typename TS>
hipError_t launch_batch_persistent(const BatchInst* dev, int ninst, int total_blocks, int px, int waves, int parity,
                                   int nsteps, int* next, hipStream_t s) {
    if constexpr (sizeof(TS) == 4) {
        if (waves == 3)
            return launch_persistent_px<TS, 3>(dev, ninst, total_blocks, px, parity, nsteps, next, s);
        return launch_persistent_px<TS, 2>(dev, ninst, total_blocks, px, parity, nsteps, next, s);
    } else {
        return launch_persistent_px<TS, fused_waves<TS, 0>()>(dev, ninst, total_blocks, px, parity, nsteps, next,
                                                               s);
    }
}

template <typename TS>
hipError_t launch_moments(const StateBuf& src, const Consts& K, const OutPtrs& out, const DiagBufs& D,
                          const GuessTables* gt, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    int tx, ty, nt, nb;
    grid_of(K, tx, ty, nt, nb);
    hipError_t e = launch_face_b<TS>(src, K, D.faceB, s);
    if (e != hipSuccess) return e;
    if (gt)
        hipLaunchKernelGGL((k_moments<TS, TE, GUESS_SINGLE>), dim3(nb), dim3(TPB), 0, s, (const TS*)src.dist,
                           (const TE*)src.efield, (const double*)D.faceB, gt, K, tx, ty, nt, out, D.scratch, D.part,
                           D.nullp);
    else
        hipLaunchKernelGGL((k_moments<TS, TE, GUESS_NONE>), dim3(nb), dim3(TPB), 0, s, (const TS*)src.dist,
                           (const TE*)src.efield, (const double*)D.faceB, gt, K, tx, ty, nt, out, D.scratch, D.part,
                           D.nullp);
    hipLaunchKernelGGL(k_divb, dim3(nb), dim3(TPB), 0, s, (const double*)D.scratch, K, tx, ty, nt, D.part2);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)D.part, nt, NPART, 0, D.result);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)D.part2, nt, 1, 1, D.result + NPART);
    hipLaunchKernelGGL(k_null_reduce, dim3(1), dim3(TPB), 0, s, (const double*)D.nullp, nt,
                       (const double*)(D.scratch + 3 * K.N), (const double*)D.ez0, (const double*)D.b0,
                       D.result + NPART + 1);
    return hipGetLastError();
}

hipError_t launch_init_bmax(const InPtrs& in, const Consts& K, double* part, double* b0, hipStream_t s) {
    const int nblk = (int)((K.N + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_init_bmax, dim3(nblk), dim3(TPB), 0, s, in, K, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)part, nblk, 1, 1, b0);
    hipLaunchKernelGGL(k_sqrt1, dim3(1), dim3(64), 0, s, b0);
    return hipGetLastError();
}

hipError_t launch_face_check(const FacePtrs& in, const Consts& K, double* part, double* result, hipStream_t s) {
    const int nblk = (int)(((int64_t)K.nx * K.ny + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_face_check, dim3(nblk), dim3(TPB), 0, s, in, K, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)part, nblk, 1, 0, result);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_ghost(const FacePtrs& in, const Consts& K, const StateBuf& dst, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    const int nblk = (int)(((int64_t)K.nx * K.ny + TPB - 1) / TPB);
    hipLaunchKernelGGL((k_init_ghost<TS, TE>), dim3(nblk), dim3(TPB), 0, s, in, K, (TS*)dst.dist, (TE*)dst.efield);
    return hipGetLastError();
}

hipError_t launch_init_ref(const InPtrs& in, const Consts& K, double* part, double* result, hipStream_t s) {
    const int nblk = (int)((K.N + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_init_ref, dim3(nblk), dim3(TPB), 0, s, in, K, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)part, nblk, 2, 0, result);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_init(const InPtrs& in, const Consts& K, double* scr, const StateBuf& dst, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    int tx, ty, nt, nb;
    grid_of(K, tx, ty, nt, nb);
    hipLaunchKernelGGL(k_init_current, dim3(nb), dim3(TPB), 0, s, in, K, tx, ty, nt, scr);
    hipLaunchKernelGGL((k_init_state<TS, TE>), dim3(nb), dim3(TPB), 0, s, in, K, tx, ty, nt, (const double*)scr,
                       (TS*)dst.dist, (TE*)dst.efield);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_export(const StateBuf& src, double* dst, const Consts& K, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    const int64_t total = K.N * state_arrays(K);
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL((k_export<TS, TE>), dim3((unsigned)blocks), dim3(256), 0, s, (const TS*)src.dist,
                       (const TE*)src.efield, dst, K);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_import(const double* src, const StateBuf& dst, const Consts& K, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    const int64_t total = K.N * state_arrays(K);
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL((k_import<TS, TE>), dim3((unsigned)blocks), dim3(256), 0, s, src, (TS*)dst.dist,
                       (TE*)dst.efield, K);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_guess_samples(const StateBuf& src, const Consts& K, double* faceB, int ns, double* F, double* T,
                                double* part, double* result, hipStream_t s) {
    using TE = typename StoreTypes<TS>::E;
    hipError_t e = launch_face_b<TS>(src, K, faceB, s);
    if (e != hipSuccess) return e;
    const int nblk = (ns + 255) / 256;
    hipLaunchKernelGGL((k_guess_samples<TS, TE>), dim3(nblk), dim3(256), 0, s, (const TS*)src.dist,
                       (const TE*)src.efield, (const double*)faceB, K, ns, F, T, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, (const double*)part, nblk, SAMPLE_SUMS, 0, result);
    return hipGetLastError();
}

#define RMHD_INSTANTIATE(TS)                                                                                          \
    template hipError_t launch_step<TS>(const StateBuf&, const StateBuf&, const Consts&, const StepTuning&, double*,  \
                                        const GuessTables*, hipStream_t);                                             \
    template hipError_t launch_moments<TS>(const StateBuf&, const Consts&, const OutPtrs&, const DiagBufs&,           \
                                           const GuessTables*, hipStream_t);                                          \
    template hipError_t launch_init<TS>(const InPtrs&, const Consts&, double*, const StateBuf&, hipStream_t);         \
    template hipError_t launch_ghost<TS>(const FacePtrs&, const Consts&, const StateBuf&, hipStream_t);               \
    template hipError_t launch_batch<TS>(const BatchInst*, int, int, int64_t, int, int, int, hipStream_t);            \
    template hipError_t launch_batch_persistent<TS>(const BatchInst*, int, int, int, int, int, int, int*,            \
                                                    hipStream_t);                                                     \
    template hipError_t launch_guess_samples<TS>(const StateBuf&, const Consts&, double*, int, double*, double*,      \
                                                 double*, double*, hipStream_t);                                      \
    template hipError_t launch_export<TS>(const StateBuf&, double*, const Consts&, hipStream_t);                      \
    template hipError_t launch_import<TS>(const double*, const StateBuf&, const Consts&, hipStream_t);

RMHD_INSTANTIATE(double)
RMHD_INSTANTIATE(float)
RMHD_INSTANTIATE(_Float16)

}  // namespace rmhd
