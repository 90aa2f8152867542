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

// Stores of the next state are never read again in this step: the
// non-temporal hint keeps them from evicting the stencil lines from L2.
template <bool NT, typename T>
__device__ __forceinline__ void st(T* __restrict__ p, double v) {
    if constexpr (NT)
        __builtin_nontemporal_store(static_cast<T>(v), p);
    else
        *p = static_cast<T>(v);
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

// Moments and macroscopic solution of one cell in one step.
struct CellSol {
    double T00, T0[3], Tab[6], N0;   // moments (Tab: xx, yy, zz, xy, xz, yz)
    double Ep[3], B[3], rho, rho_g;  // previous E, this step's B, charge, Gauss charge
    double Epr[3];                   // E' of Eq. Cal_E
    double eps, p, n, gam, beta[3], E[3], J[3];
    int iters;
    bool ok;
};

// ... plus the transported f, g and streamed h (one thread per cell).
struct Macro : CellSol {
    double F[Q], G[Q], H[QH + 1];
};

// Recovery and the Ohm-coupled E, J of one cell from its moments (M.T00,
// M.T0, M.Tab, M.N0, M.Epr, M.B, M.Ep, M.rho_g): fills eps, p, n, gam, beta,
// E, J, iters, ok.
__device__ __forceinline__ void solve_cell(const Consts& K, CellSol& M) {
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

    solve_cell(K, M);
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

// f_eq of direction sgn * e_I (sgn = +-1): the odd terms change sign, the
// weight is that of e_I.
template <int I>
__device__ __forceinline__ double feq_signed(const FeqCell& f, double sgn) {
    constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
    const double eb = sgn * (ex * f.beta[0] + ey * f.beta[1] + ez * f.beta[2]);
    const double cross =
        (ex * ey) * f.beta[0] * f.beta[1] + (ex * ez) * f.beta[0] * f.beta[2] + (ey * ez) * f.beta[1] * f.beta[2];
    const double diag = (ex * ex) * f.beta[0] * f.beta[0] + (ey * ey) * f.beta[1] * f.beta[1] +
                        (ez * ez) * f.beta[2] * f.beta[2];
    const double fluid =
        f.A1 + 19.0 * f.g2 * cross + 4.0 * KAPPA * f.g2 * eb + (4.0 / 15.0) * f.g2 * (19.0 * diag - 4.0 * f.b2);
    const double Be = ex * f.cB[0] + ey * f.cB[1] + ez * f.cB[2];
    const double Ee = ex * f.E[0] + ey * f.E[1] + ez * f.E[2];
    const double BxEe = sgn * (ex * f.BxE[0] + ey * f.BxE[1] + ez * f.BxE[2]);
    const double crossEB = (ex * ey) * (f.E[0] * f.E[1] + f.cB[0] * f.cB[1]) +
                           (ex * ez) * (f.E[0] * f.E[2] + f.cB[0] * f.cB[2]) +
                           (ey * ez) * (f.E[1] * f.E[2] + f.cB[1] * f.cB[2]);
    const double em = 2.3 * f.X - SQRT19_3 * BxEe - 3.8 * (Be * Be + Ee * Ee) - 6.65 * crossEB;
    return weight(I) * (f.P34 * fluid + f.eps0 * em);
}

template <int I, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    if constexpr (I < Q) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1>(fn);
    }
}

// Collisions and the stores of one cell (second half of the step).
template <bool NT, typename T>
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
        st<NT>(dst + (int64_t)(OFF_F + i) * K.stride + cell, M.F[i] - om * (M.F[i] - feq));
        // g: Eq. Hupp equilibrium, collision with g(t + dt) in closed form
        const double wpi = i == 0 ? K.wp[0] : (i <= 6 ? K.wp[1] : K.wp[2]);
        const double geq = wpi * M.n * M.gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * fe.b2);
        st<NT>(dst + (int64_t)(OFF_G + i) * K.stride + cell, (M.G[i] + K.wg * geq) / (1.0 + K.wg));
    });
    // h_eq of Eq. Maxwell-eq with the current coefficient 1/(32 c^2):
    // v.J / (32 c^2) = s.J / (16 sqrt2 c), E.e / (8 c^2) = ehat.E / (8 sqrt2 c), B.b / 8 = bhat.B / 8
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * K.c), ce = 1.0 / (8.0 * 1.4142135623730951 * K.c);
#pragma unroll
    for (int k = 0; k < QH; ++k) {
        const double heq = cj * (SX[k] * M.J[0] + SY[k] * M.J[1] + SZ[k] * M.J[2]) +
                           ce * (EHX[k] * M.E[0] + EHY[k] * M.E[1] + EHZ[k] * M.E[2]) +
                           0.125 * (BHX[k] * M.B[0] + BHY[k] * M.B[1] + BHZ[k] * M.B[2]);
        st<NT>(dst + (int64_t)(OFF_H + k) * K.stride + cell, 2.0 * heq - M.H[k]);  // tau_h = 1/2
    }
    st<NT>(dst + (int64_t)(OFF_H + QH) * K.stride + cell, 2.0 * M.rho - M.H[QH]);
#pragma unroll
    for (int a = 0; a < 3; ++a) st<NT>(dst + (int64_t)(OFF_E + a) * K.stride + cell, M.E[a]);
}

// ---------------------------------------------------- two lanes per cell

// The fused step with the populations of one cell split over an adjacent
// lane pair (h = lane & 1).  Slot s = 1..9 of f and g is direction 2s-1+h,
// i.e. sgn * e_{2s-1} with sgn = +1 / -1, so both lanes run the same
// instructions on opposite directions; slot m = 0..11 of h is population
// 2m+h (same streaming offset, opposite e and b).  Lane 0 also owns the rest
// populations f_0, g_0; lane 1 owns h_rest.  Partial moments are summed over
// the pair with one xor-1 shuffle each, and both lanes then run the recovery
// and the Ohm solve on identical inputs.
constexpr int PX = 64, PY = 2, PTPB = 2 * PX * PY;

__device__ __forceinline__ double pair_sum(double v) { return v + __shfl_xor(v, 1, 64); }

template <bool NT, typename T>
__device__ __forceinline__ void pair_cell(const T* __restrict__ src, T* __restrict__ dst, const Consts& K, int cell,
                                          const Nbr& nb, int h) {
    const double sgn = h ? -1.0 : 1.0;
    const int64_t S = K.stride;
    // Array bases stay uniform (scalar registers); the lane's choice between
    // the two arrays of a pair is folded into its 32-bit element index.
    const int hc = cell + (h ? (int)S : 0);
    double Fv[10], Gv[10], Hv[13];
    double t00 = 0, t0x = 0, t0y = 0, t0z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0, n0 = 0;
    // slot 0: f_0, g_0 (lane 0) and h_rest (lane 1)
    {
        const double a = ld(src + (h ? (int64_t)(OFF_H + QH) : (int64_t)OFF_F) * S + cell, 0);
        const double g = ld(src + (int64_t)OFF_G * S + cell, 0);
        Fv[0] = h ? 0.0 : a;
        Gv[0] = h ? 0.0 : g;
        Hv[12] = h ? a : 0.0;
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
            const T* __restrict__ fa = src + (int64_t)(OFF_F + i0) * S;
            const T* __restrict__ ga = src + (int64_t)(OFF_G + i0) * S;
            const double f0 = ld(fa, hc), fm2 = ld(fa, hc + om2), fm1 = ld(fa, hc + om1), fp1 = ld(fa, hc + op1);
            const double lap = (ld(fa, hc + lap_xp) + ld(fa, hc + lap_xm)) + (ld(fa, hc + lap_yp) + ld(fa, hc + lap_ym)) +
                               (ld(fa, hc + lap_zp) + ld(fa, hc + lap_zm)) - 6.0 * f0;
            const double fv = f0 - K.cour * ((f0 + 0.5 * minmod(f0 - fm1, fp1 - f0)) -
                                             (fm1 + 0.5 * minmod(fm1 - fm2, f0 - fm1))) + K.kv * lap;
            const double g0 = ld(ga, hc), gm2 = ld(ga, hc + om2), gm1 = ld(ga, hc + om1), gp1 = ld(ga, hc + op1);
            const double gv = g0 - K.cour * ((g0 + 0.5 * minmod(g0 - gm1, gp1 - g0)) -
                                             (gm1 + 0.5 * minmod(gm1 - gm2, g0 - gm1)));
            Fv[s] = fv;
            Gv[s] = gv;
            // Keep each slot's arithmetic next to its loads: without this the
            // scheduler sinks all of it below every load of the cell, and the
            // ~150 load destinations in flight cost a wave its occupancy.
            asm volatile("" : "+v"(Fv[s]), "+v"(Gv[s])::"memory");
            t00 += fv;
            n0 += gv;
            const double sf = sgn * fv;
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
    double ehx = 0, ehy = 0, ehz = 0, bx = 0, by = 0, bz = 0, hs = 0;
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const double v = ld(src + (int64_t)(OFF_H + k0) * S, hc + nb.at(-SX[k0], -SY[k0], -SZ[k0]));
        Hv[m] = v;
        hs += v;
        const double sv = sgn * v;
        if (EHX[k0]) ehx += EHX[k0] * sv;
        if (EHY[k0]) ehy += EHY[k0] * sv;
        if (EHZ[k0]) ehz += EHZ[k0] * sv;
        if (BHX[k0]) bx += BHX[k0] * sv;
        if (BHY[k0]) by += BHY[k0] * sv;
        if (BHZ[k0]) bz += BHZ[k0] * sv;
    }
    CellSol M;
#pragma unroll
    for (int a = 0; a < 3; ++a) M.Ep[a] = ld(src + (int64_t)(OFF_E + a) * S + cell, 0);
    // Gauss charge: lane 0 takes E_x(x+-1), E_y(y+1); lane 1 E_y(y-1), E_z(z+-1)
    double gpart;
    {
        const T* ex_ = src + (int64_t)(OFF_E + 0) * S + cell;
        const T* ey_ = src + (int64_t)(OFF_E + 1) * S + cell;
        const T* ez_ = src + (int64_t)(OFF_E + 2) * S + cell;
        const double a = h ? -ld(ey_, lap_ym) : ld(ex_, lap_xp);
        const double b = h ? ld(ez_, lap_zp) : -ld(ex_, lap_xm);
        const double c = h ? -ld(ez_, lap_zm) : ld(ey_, lap_yp);
        gpart = (a + b) + c;
    }
    M.T00 = pair_sum(t00);
    M.N0 = pair_sum(n0);
    M.T0[0] = KAPPA * pair_sum(t0x);
    M.T0[1] = KAPPA * pair_sum(t0y);
    M.T0[2] = KAPPA * pair_sum(t0z);
    M.Tab[0] = KAPPA2 * pair_sum(txx);
    M.Tab[1] = KAPPA2 * pair_sum(tyy);
    M.Tab[2] = KAPPA2 * pair_sum(tzz);
    M.Tab[3] = KAPPA2 * pair_sum(txy);
    M.Tab[4] = KAPPA2 * pair_sum(txz);
    M.Tab[5] = KAPPA2 * pair_sum(tyz);
    const double ec = K.c * INV_SQRT2;
    M.Epr[0] = ec * pair_sum(ehx);
    M.Epr[1] = ec * pair_sum(ehy);
    M.Epr[2] = ec * pair_sum(ehz);
    M.B[0] = pair_sum(bx);
    M.B[1] = pair_sum(by);
    M.B[2] = pair_sum(bz);
    M.rho = pair_sum(Hv[12] + hs);
    M.rho_g = K.eps0 * K.inv_2dx * pair_sum(gpart);
    solve_cell(K, M);

    // collisions and stores
    FeqCell fe;
    fe.setup(M.eps, M.p, M.gam, M.beta, M.Ep, M.B, K.c, K.eps0);
    const double rate = M.gam * K.inv_tau;
    const double inv1wg = 1.0 / (1.0 + K.wg);
    if (h == 0) {
        const double feq0 = fe.eq<0>();
        st<NT>(dst + (int64_t)OFF_F * S + cell, Fv[0] - rate * (Fv[0] - feq0));
        const double geq0 = K.wp[0] * M.n * M.gam * (1.0 - K.gc3 * fe.b2);
        st<NT>(dst + (int64_t)OFF_G * S + cell, (Gv[0] + K.wg * geq0) * inv1wg);
    } else {
        st<NT>(dst + (int64_t)(OFF_H + QH) * S + cell, 2.0 * M.rho - Hv[12]);
    }
    static_for<1>([&](auto ic) {
        constexpr int s = decltype(ic)::value;
        if constexpr (s <= 9) {
            constexpr int i0 = 2 * s - 1;
            const double eb = sgn * (EX[i0] * M.beta[0] + EY[i0] * M.beta[1] + EZ[i0] * M.beta[2]);
            const double om = rate * (1.0 - KAPPA * eb);
            const double feq = feq_signed<i0>(fe, sgn);
            st<NT>(dst + (int64_t)(OFF_F + i0) * S + hc, Fv[s] - om * (Fv[s] - feq));
            const double wpi = i0 <= 6 ? K.wp[1] : K.wp[2];
            const double geq = wpi * M.n * M.gam * (1.0 + K.gc1 * eb + K.gc2 * eb * eb - K.gc3 * fe.b2);
            st<NT>(dst + (int64_t)(OFF_G + i0) * S + hc, (Gv[s] + K.wg * geq) * inv1wg);
        }
    });
    const double cj = 1.0 / (16.0 * 1.4142135623730951 * K.c), ce = 1.0 / (8.0 * 1.4142135623730951 * K.c);
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const int k0 = 2 * m;
        const double heq = cj * (SX[k0] * M.J[0] + SY[k0] * M.J[1] + SZ[k0] * M.J[2]) +
                           sgn * (ce * (EHX[k0] * M.E[0] + EHY[k0] * M.E[1] + EHZ[k0] * M.E[2]) +
                                  0.125 * (BHX[k0] * M.B[0] + BHY[k0] * M.B[1] + BHZ[k0] * M.B[2]));
        st<NT>(dst + (int64_t)(OFF_H + k0) * S + hc, 2.0 * heq - Hv[m]);
    }
    if (h == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) st<NT>(dst + (int64_t)(OFF_E + a) * S + cell, M.E[a]);
    }
}

// ------------------------------------------------------------------ kernels

// One block owns a 64 x 4 column tile and walks zb consecutive z-planes.
// Blocks are numbered column-fastest within a z-chunk, and XCD k receives the
// contiguous block range [k P, (k + 1) P): the columns one XCD runs at the same
// time are neighbours marching through the same planes, so the y-halo and the
// z-neighbour planes of the stencil are shared in that XCD's L2.
template <bool NT, typename T>
__global__ __launch_bounds__(TPB) void k_fused_step(const T* __restrict__ src, T* __restrict__ dst, Consts K,
                                                    int tiles_x, int ncol, int zb, int nblk) {
    const int b = tile_of_block(nblk);
    if (b >= nblk) return;
    const int col = b % ncol, zc = b / ncol;
    const int tx = col % tiles_x, ty = col / tiles_x;
    const int x = tx * TX + (threadIdx.x % TX), y = ty * TY + (threadIdx.x / TX);
    if (x >= K.nx || y >= K.ny) return;
    const int z0 = zc * zb, z1 = min(K.nz, z0 + zb);
    for (int z = z0; z < z1; ++z) {
        const int cell = x + K.nx * (y + K.ny * z);
        const Nbr nb = make_nbr(K, x, y, z);
        Macro M;
        macroscopic(src, K, cell, nb, M);
        collide_store<NT>(dst, K, cell, M);
    }
}

template <bool NT, typename T>
__global__ __launch_bounds__(PTPB, 2) void k_fused_step_pair(const T* __restrict__ src, T* __restrict__ dst, Consts K,
                                                          int tiles_x, int ncol, int zb, int nblk) {
    const int b = tile_of_block(nblk);
    if (b >= nblk) return;
    const int col = b % ncol, zc = b / ncol;
    const int tx = col % tiles_x, ty = col / tiles_x;
    const int c = threadIdx.x >> 1, h = threadIdx.x & 1;
    const int x = tx * PX + (c % PX), y = ty * PY + c / PX;
    if (x >= K.nx || y >= K.ny) return;  // both lanes of a pair leave together
    const int z0 = zc * zb, z1 = min(K.nz, z0 + zb);
    for (int z = z0; z < z1; ++z) {
        const int cell = x + K.nx * (y + K.ny * z);
        const Nbr nb = make_nbr(K, x, y, z);
        pair_cell<NT>(src, dst, K, cell, nb, h);
    }
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
hipError_t launch_step(const void* src, void* dst, const Consts& K, const StepTuning& tune, hipStream_t s) {
    const int tiles_x = (K.nx + TX - 1) / TX, tiles_y = (K.ny + TY - 1) / TY;
    const int zb = tune.zb > 0 ? (tune.zb < K.nz ? tune.zb : K.nz) : 1;
    const int ncol = tiles_x * tiles_y, nblk = ncol * ((K.nz + zb - 1) / zb);
    const int grid = ((nblk + 7) / 8) * 8;
    if (tune.pair) {
        const int ptx = (K.nx + PX - 1) / PX, pcol = ptx * ((K.ny + PY - 1) / PY);
        const int pblk = pcol * ((K.nz + zb - 1) / zb), pgrid = ((pblk + 7) / 8) * 8;
        if (tune.nt_store)
            hipLaunchKernelGGL((k_fused_step_pair<true, T>), dim3(pgrid), dim3(PTPB), 0, s, (const T*)src, (T*)dst, K,
                               ptx, pcol, zb, pblk);
        else
            hipLaunchKernelGGL((k_fused_step_pair<false, T>), dim3(pgrid), dim3(PTPB), 0, s, (const T*)src, (T*)dst,
                               K, ptx, pcol, zb, pblk);
        return hipGetLastError();
    }
    if (tune.nt_store)
        hipLaunchKernelGGL((k_fused_step<true, T>), dim3(grid), dim3(TPB), 0, s, (const T*)src, (T*)dst, K, tiles_x,
                           ncol, zb, nblk);
    else
        hipLaunchKernelGGL((k_fused_step<false, T>), dim3(grid), dim3(TPB), 0, s, (const T*)src, (T*)dst, K, tiles_x,
                           ncol, zb, nblk);
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

template hipError_t launch_step<double>(const void*, void*, const Consts&, const StepTuning&, hipStream_t);
template hipError_t launch_step<float>(const void*, void*, const Consts&, const StepTuning&, hipStream_t);
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
