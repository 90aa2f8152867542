// rmhdlb_kernels.hip -- gfx950 kernels of the resistive relativistic MHD
// lattice Boltzmann step (arXiv:1508.03452, Sec. III).
//
// Layout in HBM: structure of arrays, one array per population, x fastest:
//   state[a * stride + cell], a = F[0..18], G[0..18], h*[0..24], E_prev[0..2],
// two such buffers (read one, write the other).  The stored state is
// post-collision.  One thread owns one cell; a 64 x 4 tile of cells is one
// workgroup (one wavefront per x-row of 64, so every load of an array row is
// one coalesced 512-byte FP64 segment).  Tiles are handed out so that each of
// the 8 XCDs works on a contiguous slab of the grid and the stencil
// neighbours of its tiles stay in that XCD's L2.
#include "rmhdlb_device.h"
#include "rmhdlb_internal.h"

namespace rmhd {

constexpr int TX = 64, TY = 4, TPB = TX * TY;

template <typename T>
__device__ __forceinline__ double ld(const T* __restrict__ p, int64_t i) {
    return static_cast<double>(p[i]);
}

// Neighbour offsets of one cell along one axis for displacements -2..+2,
// with periodic wrap or (open face) a copy of the first interior cell.
__device__ __forceinline__ int map_coord(int v, int n, int periodic) {
    if (v < 0) return periodic ? (v + n >= 0 ? v + n : v + 2 * n) : 0;
    if (v >= n) return periodic ? (v - n < n ? v - n : v - 2 * n) : n - 1;
    return v;
}

struct Nbr {
    int ox[5], oy[5], oz[5];  // element offsets for displacement d = -2..2 (index d + 2)
    __device__ __forceinline__ int at(int dx, int dy, int dz) const { return ox[dx + 2] + oy[dy + 2] + oz[dz + 2]; }
};

__device__ __forceinline__ Nbr make_nbr(const Consts& K, int x, int y, int z) {
    Nbr n;
    const int sy = K.nx, sz = K.nx * K.ny;
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        n.ox[d + 2] = map_coord(x + d, K.nx, K.per[0]) - x;
        n.oy[d + 2] = (map_coord(y + d, K.ny, K.per[1]) - y) * sy;
        n.oz[d + 2] = (map_coord(z + d, K.nz, K.per[2]) - z) * sz;
    }
    return n;
}

// Tile index with XCD-aware placement: block b runs on XCD b % 8, so XCD k is
// given the contiguous tile range [k P, (k + 1) P).
__device__ __forceinline__ int tile_of_block(int nblocks) {
    const int P = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * P + blockIdx.x / 8;
}

// Per-cell macroscopic state of one step.
struct Macro {
    double F[Q], G[Q], H[QH + 1];  // transported f, g and streamed h
    double T00, T0[3], Tab[6], N0;  // moments (Tab: xx, yy, zz, xy, xz, yz)
    double Ep[3], B[3], rho, rho_g;  // previous E, this step's B, charge, Gauss charge
    double Epr[3];                  // E' of Eq. Cal_E
    double eps, p, n, gam, beta[3], E[3], J[3];
    int iters;
    bool ok;
};

// Transport (collide-then-transport reading of Eq. rlb): link-wise
// minmod-MUSCL flux difference, plus the 7-point bulk-viscosity Laplacian
// for i != 0; g without viscosity.  Then the streaming of h, the moments,
// the recovery and E, J.
template <typename T>
__device__ __forceinline__ void macroscopic(const T* __restrict__ src, const Consts& K, int cell, const Nbr& nb,
                                            Macro& M) {
    M.T00 = 0.0;
    M.N0 = 0.0;
    double t0x = 0, t0y = 0, t0z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T* __restrict__ fa = src + (int64_t)(OFF_F + i) * K.stride + cell;
        const T* __restrict__ ga = src + (int64_t)(OFF_G + i) * K.stride + cell;
        const double f0 = ld(fa, 0), g0 = ld(ga, 0);
        double fv = f0, gv = g0;
        if (i != 0) {
            const int ex = EX[i], ey = EY[i], ez = EZ[i];
            const int om2 = nb.at(-2 * ex, -2 * ey, -2 * ez), om1 = nb.at(-ex, -ey, -ez), op1 = nb.at(ex, ey, ez);
            {
                const double fm2 = ld(fa, om2), fm1 = ld(fa, om1), fp1 = ld(fa, op1);
                const double face_p = f0 + 0.5 * minmod(f0 - fm1, fp1 - f0);
                const double face_m = fm1 + 0.5 * minmod(fm1 - fm2, f0 - fm1);
                const double lap = (ld(fa, nb.at(1, 0, 0)) + ld(fa, nb.at(-1, 0, 0))) +
                                   (ld(fa, nb.at(0, 1, 0)) + ld(fa, nb.at(0, -1, 0))) +
                                   (ld(fa, nb.at(0, 0, 1)) + ld(fa, nb.at(0, 0, -1))) - 6.0 * f0;
                fv = f0 - K.cour * (face_p - face_m) + K.kv * lap;
            }
            {
                const double gm2 = ld(ga, om2), gm1 = ld(ga, om1), gp1 = ld(ga, op1);
                const double face_p = g0 + 0.5 * minmod(g0 - gm1, gp1 - g0);
                const double face_m = gm1 + 0.5 * minmod(gm1 - gm2, g0 - gm1);
                gv = g0 - K.cour * (face_p - face_m);
            }
        }
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
        const T* __restrict__ ha = src + (int64_t)(OFF_H + k) * K.stride + cell;
        const double h = ld(ha, nb.at(-SX[k], -SY[k], -SZ[k]));
        M.H[k] = h;
        hs += h;
        if (EHX[k]) ehx += EHX[k] * h;
        if (EHY[k]) ehy += EHY[k] * h;
        if (EHZ[k]) ehz += EHZ[k] * h;
        if (BHX[k]) bx += BHX[k] * h;
        if (BHY[k]) by += BHY[k] * h;
        if (BHZ[k]) bz += BHZ[k] * h;
    }
    M.H[QH] = ld(src + (int64_t)(OFF_H + QH) * K.stride + cell, 0);
    const double ec = K.c * INV_SQRT2;  // |e_k| / |ehat_k|
    M.Epr[0] = ec * ehx;
    M.Epr[1] = ec * ehy;
    M.Epr[2] = ec * ehz;
    M.B[0] = bx;
    M.B[1] = by;
    M.B[2] = bz;
    M.rho = M.H[QH] + hs;

    // previous E and its Gauss charge
    const T* __restrict__ e0 = src + (int64_t)(OFF_E + 0) * K.stride + cell;
    const T* __restrict__ e1 = src + (int64_t)(OFF_E + 1) * K.stride + cell;
    const T* __restrict__ e2 = src + (int64_t)(OFF_E + 2) * K.stride + cell;
    M.Ep[0] = ld(e0, 0);
    M.Ep[1] = ld(e1, 0);
    M.Ep[2] = ld(e2, 0);
    M.rho_g = K.eps0 * K.inv_2dx *
              ((ld(e0, nb.at(1, 0, 0)) - ld(e0, nb.at(-1, 0, 0))) + (ld(e1, nb.at(0, 1, 0)) - ld(e1, nb.at(0, -1, 0))) +
               (ld(e2, nb.at(0, 0, 1)) - ld(e2, nb.at(0, 0, -1))));

    // fluid tensor with E_prev and this step's B
    const double c = K.c, c2 = c * c;
    const double* E = M.Ep;
    const double* B = M.B;
    const double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    const double U = 0.5 * (E2 + c2 * B2);
    const double Ef = M.T00 - K.eps0 * U;
    double S[3], Pi[6];
    S[0] = M.T0[0] - K.eps0 * c * (E[1] * B[2] - E[2] * B[1]);
    S[1] = M.T0[1] - K.eps0 * c * (E[2] * B[0] - E[0] * B[2]);
    S[2] = M.T0[2] - K.eps0 * c * (E[0] * B[1] - E[1] * B[0]);
    Pi[0] = M.Tab[0] - K.eps0 * (U - E[0] * E[0] - c2 * B[0] * B[0]);
    Pi[1] = M.Tab[1] - K.eps0 * (U - E[1] * E[1] - c2 * B[1] * B[1]);
    Pi[2] = M.Tab[2] - K.eps0 * (U - E[2] * E[2] - c2 * B[2] * B[2]);
    Pi[3] = M.Tab[3] + K.eps0 * (E[0] * E[1] + c2 * B[0] * B[1]);
    Pi[4] = M.Tab[4] + K.eps0 * (E[0] * E[2] + c2 * B[0] * B[2]);
    Pi[5] = M.Tab[5] + K.eps0 * (E[1] * E[2] + c2 * B[1] * B[2]);

    double lam;
    M.iters = recover(Ef, S, Pi, lam, M.beta);
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

// f_eq of Eq. Dis_fun_EM in normalised variables (F = (c_t/c_0)^2 f), with
// the corrections that make its moments T_fluid + T_EM: the delta_i0
// coefficient 361 (3p - eps) / (33 (p + eps)), the minus sign of the
// (E.c_i)^2 term, the y-z cross terms, and c on the (B x E).c_i term.
struct FeqCell {
    double P34, A1, Bc, g2, beta[3], b2, eps0;
    double X, BxE[3], E[3], cB[3];
    __device__ __forceinline__ void setup(double eps, double p, double gam, const double bta[3], const double Ev[3],
                                          const double Bv[3], double c, double e0) {
        P34 = 0.75 * (eps + p);
        A1 = 1.0 + (3.0 * p - eps) / (p + eps);
        Bc = 361.0 * (3.0 * p - eps) / (33.0 * (p + eps));
        g2 = gam * gam;
        b2 = bta[0] * bta[0] + bta[1] * bta[1] + bta[2] * bta[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            beta[a] = bta[a];
            E[a] = Ev[a];
            cB[a] = c * Bv[a];
        }
        X = cB[0] * cB[0] + cB[1] * cB[1] + cB[2] * cB[2] + E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
        // c (B x E)
        BxE[0] = cB[1] * E[2] - cB[2] * E[1];
        BxE[1] = cB[2] * E[0] - cB[0] * E[2];
        BxE[2] = cB[0] * E[1] - cB[1] * E[0];
        eps0 = e0;
    }
    template <int I>
    __device__ __forceinline__ double eq() const {
        constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
        const double eb = ex * beta[0] + ey * beta[1] + ez * beta[2];
        const double cross = (ex * ey) * beta[0] * beta[1] + (ex * ez) * beta[0] * beta[2] + (ey * ez) * beta[1] * beta[2];
        const double diag = (ex * ex) * beta[0] * beta[0] + (ey * ey) * beta[1] * beta[1] + (ez * ez) * beta[2] * beta[2];
        double fluid = A1 + 19.0 * g2 * cross + 4.0 * KAPPA * g2 * eb + (4.0 / 15.0) * g2 * (19.0 * diag - 4.0 * b2);
        if (I == 0) fluid += Bc;
        const double Be = ex * cB[0] + ey * cB[1] + ez * cB[2];
        const double Ee = ex * E[0] + ey * E[1] + ez * E[2];
        const double BxEe = ex * BxE[0] + ey * BxE[1] + ez * BxE[2];
        const double crossEB = (ex * ey) * (E[0] * E[1] + cB[0] * cB[1]) + (ex * ez) * (E[0] * E[2] + cB[0] * cB[2]) +
                               (ey * ez) * (E[1] * E[2] + cB[1] * cB[2]);
        const double em = 2.3 * X - SQRT19_3 * BxEe - 3.8 * (Be * Be + Ee * Ee) - 6.65 * crossEB;
        return weight(I) * (P34 * fluid + eps0 * em);
    }
};

template <int I, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    if constexpr (I < Q) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1>(fn);
    }
}

// Collisions and the stores of one cell (second half of the step).
template <typename T>
__device__ __forceinline__ void collide_store(T* __restrict__ dst, const Consts& K, int cell, const Macro& M) {
    FeqCell fe;
    // Reading of the coupling: f_eq carries T_EM of the same pair (E_prev, B)
    // that the recovery subtracted, so the collision conserves T^{0 nu}.
    fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, M.B, K.c, K.eps0);
    const double rate = M.gam * K.inv_tau;
    static_for<0>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double eb = EX[i] * M.beta[0] + EY[i] * M.beta[1] + EZ[i] * M.beta[2];
        const double om = rate * (1.0 - KAPPA * eb);  // Anderson-Witting: gamma (1 - kappa e.beta) / tau
        const double feq = fe.eq<i>();
        dst[(int64_t)(OFF_F + i) * K.stride + cell] = static_cast<T>(M.F[i] - om * (M.F[i] - feq));
        // g: Eq. Hupp equilibrium, collision with g(t + dt) in closed form
        const double wpi = i == 0 ? K.wp[0] : (i <= 6 ? K.wp[1] : K.wp[2]);
        const double geq = wpi * M.n * M.gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * fe.b2);
        dst[(int64_t)(OFF_G + i) * K.stride + cell] = static_cast<T>((M.G[i] + K.wg * geq) / (1.0 + K.wg));
    });
    // h_eq of Eq. Maxwell-eq with the current coefficient 1/(32 c^2):
    // v.J / (32 c^2) = s.J / (16 sqrt2 c), E.e / (8 c^2) = ehat.E / (8 sqrt2 c), B.b / 8 = bhat.B / 8
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * K.c), ce = 1.0 / (8.0 * 1.4142135623730951 * K.c);
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const double heq = cj * (SX[k] * M.J[0] + SY[k] * M.J[1] + SZ[k] * M.J[2]) +
                           ce * (EHX[k] * M.E[0] + EHY[k] * M.E[1] + EHZ[k] * M.E[2]) +
                           0.125 * (BHX[k] * M.B[0] + BHY[k] * M.B[1] + BHZ[k] * M.B[2]);
        dst[(int64_t)(OFF_H + k) * K.stride + cell] = static_cast<T>(2.0 * heq - M.H[k]);  // tau_h = 1/2
    }
    dst[(int64_t)(OFF_H + QH) * K.stride + cell] = static_cast<T>(2.0 * M.rho - M.H[QH]);
#pragma unroll
    for (int a = 0; a < 3; ++a) dst[(int64_t)(OFF_E + a) * K.stride + cell] = static_cast<T>(M.E[a]);
}

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ __launch_bounds__(TPB) void k_fused_step(const T* __restrict__ src, T* __restrict__ dst, Consts K,
                                                    int tiles_x, int tiles_y, int ntiles) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    if (x >= K.nx || y >= K.ny) return;
    const int cell = x + K.nx * (y + K.ny * z);
    const Nbr nb = make_nbr(K, x, y, z);
    Macro M;
    macroscopic(src, K, cell, nb, M);
    collide_store(dst, K, cell, M);
}

// Primitives of the current state and per-block partial diagnostics:
// part[blk * NPART + j], j = T00, N0, T0x, T0y, T0z, em energy, rho, iters, failed.
template <typename T>
__global__ __launch_bounds__(TPB) void k_moments(const T* __restrict__ src, Consts K, int tiles_x, int tiles_y,
                                                 int ntiles, OutPtrs out, double* __restrict__ Bscratch,
                                                 double* __restrict__ part) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    double v[NPART] = {0};
    if (x < K.nx && y < K.ny) {
        const int cell = x + K.nx * (y + K.ny * z);
        const Nbr nb = make_nbr(K, x, y, z);
        Macro M;
        macroscopic(src, K, cell, nb, M);
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
            Bscratch[(int64_t)a * K.N + cell] = M.B[a];
        }
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
    }
    block_sum<NPART>(v, part + (int64_t)tile * NPART);
}

// max |div B| per block from the B field written by k_moments.
__global__ __launch_bounds__(TPB) void k_divb(const double* __restrict__ Bs, Consts K, int tiles_x, int tiles_y,
                                              int ntiles, double* __restrict__ part) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    double v[1] = {0.0};
    if (x < K.nx && y < K.ny) {
        const int cell = x + K.nx * (y + K.ny * z);
        const Nbr nb = make_nbr(K, x, y, z);
        const double* b0 = Bs + cell;
        const double* b1 = Bs + K.N + cell;
        const double* b2 = Bs + 2 * K.N + cell;
        const double dv = ((b0[nb.at(1, 0, 0)] - b0[nb.at(-1, 0, 0)]) + (b1[nb.at(0, 1, 0)] - b1[nb.at(0, -1, 0)]) +
                           (b2[nb.at(0, 0, 1)] - b2[nb.at(0, 0, -1)])) *
                          K.inv_2dx;
        v[0] = fabs(dv);
    }
    block_max1(v[0], part + tile);
}

// Fixed-order reduction of the per-block partials by one block.
__global__ __launch_bounds__(TPB) void k_reduce(const double* __restrict__ part, int nblk, int width, int is_max,
                                                double* __restrict__ out) {
    for (int j = 0; j < width; ++j) {
        double acc = is_max ? 0.0 : 0.0;
        for (int b = threadIdx.x; b < nblk; b += TPB) {
            const double v = part[(int64_t)b * width + j];
            acc = is_max ? fmax(acc, v) : acc + v;
        }
        double r = is_max ? block_max_value(acc) : block_sum_value(acc);
        if (threadIdx.x == 0) out[j] = r;
        __syncthreads();
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
    const Nbr nb = make_nbr(K, x, y, z);
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

// Initial state, pass 2: f* = f_eq, g* = g_eq, h*_k(x) = h_eq-form at x + s_k,
// h*_rest = rho_c, E_prev = E0.
template <typename T>
__global__ __launch_bounds__(TPB) void k_init_state(InPtrs in, Consts K, int tiles_x, int tiles_y, int ntiles,
                                                    const double* __restrict__ scr, T* __restrict__ dst) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % tiles_x, rest = tile / tiles_x;
    const int ty = rest % tiles_y, z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    if (x >= K.nx || y >= K.ny) return;
    const int cell = x + K.nx * (y + K.ny * z);
    const Nbr nb = make_nbr(K, x, y, z);
    const double c = K.c, c2 = c * c;
    Macro M;
    double u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = in.u[a][cell];
        M.Ep[a] = in.E[a][cell];
        M.B[a] = in.B[a][cell];
        M.beta[a] = u[a] / c;
    }
    const double n = in.n[cell], p = in.p[cell];
    const double b2 = M.beta[0] * M.beta[0] + M.beta[1] * M.beta[1] + M.beta[2] * M.beta[2];
    const double gam = 1.0 / sqrt(1.0 - b2);
    const double eps = n * c2 + p / K.gm1;
    FeqCell fe;
    fe.setup(eps, p, gam, M.beta, M.Ep, M.B, c, K.eps0);
    static_for<0>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double eb = EX[i] * M.beta[0] + EY[i] * M.beta[1] + EZ[i] * M.beta[2];
        dst[(int64_t)(OFF_F + i) * K.stride + cell] = static_cast<T>(fe.eq<i>());
        const double wpi = i == 0 ? K.wp[0] : (i <= 6 ? K.wp[1] : K.wp[2]);
        dst[(int64_t)(OFF_G + i) * K.stride + cell] =
            static_cast<T>(wpi * n * gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * b2));
    });
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * c), ce = 1.0 / (8.0 * 1.4142135623730951 * c);
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const int t = cell + nb.at(SX[k], SY[k], SZ[k]);
        const double J0 = scr[t], J1 = scr[K.N + t], J2 = scr[2 * K.N + t];
        const double P0 = scr[3 * K.N + t], P1 = scr[4 * K.N + t], P2 = scr[5 * K.N + t];
        const double heq = cj * (SX[k] * J0 + SY[k] * J1 + SZ[k] * J2) + ce * (EHX[k] * P0 + EHY[k] * P1 + EHZ[k] * P2) +
                           0.125 * (BHX[k] * in.B[0][t] + BHY[k] * in.B[1][t] + BHZ[k] * in.B[2][t]);
        dst[(int64_t)(OFF_H + k) * K.stride + cell] = static_cast<T>(heq);
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
    dst[(int64_t)(OFF_H + QH) * K.stride + cell] = static_cast<T>(rho);
#pragma unroll
    for (int a = 0; a < 3; ++a) dst[(int64_t)(OFF_E + a) * K.stride + cell] = static_cast<T>(M.Ep[a]);
}

// Raw state conversion to / from the FP64 interface layout.
template <typename T>
__global__ void k_export(const T* __restrict__ s, double* __restrict__ d, int64_t N, int64_t stride) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * NSTATE) return;
    const int64_t a = i / N, cell = i - a * N;
    d[i] = static_cast<double>(s[a * stride + cell]);
}

template <typename T>
__global__ void k_import(const double* __restrict__ s, T* __restrict__ d, int64_t N, int64_t stride) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * NSTATE) return;
    const int64_t a = i / N, cell = i - a * N;
    d[a * stride + cell] = static_cast<T>(s[i]);
}

// ------------------------------------------------------------ host launchers

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

template <typename T>
hipError_t launch_step(const void* src, void* dst, const Consts& K, hipStream_t s) {
    int tx, ty, nt, nb;
    grid_of(K, tx, ty, nt, nb);
    hipLaunchKernelGGL(k_fused_step<T>, dim3(nb), dim3(TPB), 0, s, (const T*)src, (T*)dst, K, tx, ty, nt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_moments(const void* src, const Consts& K, const OutPtrs& out, double* Bscr, double* part,
                          double* part2, double* result, hipStream_t s) {
    int tx, ty, nt, nb;
    grid_of(K, tx, ty, nt, nb);
    hipLaunchKernelGGL(k_moments<T>, dim3(nb), dim3(TPB), 0, s, (const T*)src, K, tx, ty, nt, out, Bscr, part);
    hipLaunchKernelGGL(k_divb, dim3(nb), dim3(TPB), 0, s, (const double*)Bscr, K, tx, ty, nt, part2);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)part, nt, NPART, 0, result);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, s, (const double*)part2, nt, 1, 1, result + NPART);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const InPtrs& in, const Consts& K, double* scr, void* dst, hipStream_t s) {
    int tx, ty, nt, nb;
    grid_of(K, tx, ty, nt, nb);
    hipLaunchKernelGGL(k_init_current, dim3(nb), dim3(TPB), 0, s, in, K, tx, ty, nt, scr);
    hipLaunchKernelGGL(k_init_state<T>, dim3(nb), dim3(TPB), 0, s, in, K, tx, ty, nt, (const double*)scr, (T*)dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const void* src, double* dst, const Consts& K, hipStream_t s) {
    const int64_t total = K.N * NSTATE;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_export<T>, dim3((unsigned)blocks), dim3(256), 0, s, (const T*)src, dst, K.N, K.stride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_import(const double* src, void* dst, const Consts& K, hipStream_t s) {
    const int64_t total = K.N * NSTATE;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_import<T>, dim3((unsigned)blocks), dim3(256), 0, s, src, (T*)dst, K.N, K.stride);
    return hipGetLastError();
}

template hipError_t launch_step<double>(const void*, void*, const Consts&, hipStream_t);
template hipError_t launch_step<float>(const void*, void*, const Consts&, hipStream_t);
template hipError_t launch_moments<double>(const void*, const Consts&, const OutPtrs&, double*, double*, double*,
                                           double*, hipStream_t);
template hipError_t launch_moments<float>(const void*, const Consts&, const OutPtrs&, double*, double*, double*,
                                          double*, hipStream_t);
template hipError_t launch_init<double>(const InPtrs&, const Consts&, double*, void*, hipStream_t);
template hipError_t launch_init<float>(const InPtrs&, const Consts&, double*, void*, hipStream_t);
template hipError_t launch_export<double>(const void*, double*, const Consts&, hipStream_t);
template hipError_t launch_export<float>(const void*, double*, const Consts&, hipStream_t);
template hipError_t launch_import<double>(const double*, void*, const Consts&, hipStream_t);
template hipError_t launch_import<float>(const double*, void*, const Consts&, hipStream_t);

}  // namespace rmhd
