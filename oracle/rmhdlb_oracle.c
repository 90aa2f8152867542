/*
 * rmhdlb_oracle.c -- oracle for the lattice Boltzmann model of resistive
 * relativistic magnetohydrodynamics (Mohseni, Mendoza, Succi, Herrmann,
 * arXiv:1508.03452, Sec. III).
 *
 * TEST INFRASTRUCTURE.  This is a plain, slow, single-threaded FP64
 * implementation of the method's time step, written from the paper in the
 * paper's own variables (f, g, h, xi^mu, chi^mu, c_a, c_t/c_0, nu).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it; the HIP library never does.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (see oracle/build.py).
 *
 * Every place where the paper is silent, garbled or inconsistent with itself
 * is marked "Reading Rn" with the reading taken and the reason for it.
 *
 * Loop order is fixed: cells in x-fastest order, directions in table order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ERECOVERY -4
#define ORC_EUNSUPPORTED -5

#define BC_PERIODIC 0
#define BC_OPEN 1
#define BC_DRIVEN 2 /* low face of z only: fixed ghost planes (Reading R23) */

#define Q19 19
#define QH 24 /* moving Maxwell populations; index 24 is the rest population */
#define NSTATE (Q19 + Q19 + QH + 1 + 3)

typedef struct {
    int32_t nx, ny, nz;
    int32_t bc_lo[3], bc_hi[3]; /* 0 periodic, 1 open */
    double dx, c, mu0;
    double tau;   /* fluid relaxation time in units of dt (Reading R3) */
    double tau_h; /* Maxwell relaxation time, must be 1/2 (Eq. Ex_force) */
    double alpha, Gamma, sigma, nu;
    int32_t divb_fix;  /* normal-B adjustment on open faces (Reading R22) */
    int32_t null_band; /* half-width in y-cells of the null-point search band (< 1: 64) */
    int32_t collision; /* f collision: 0 explicit (Reading R4), 1 the printed semi-implicit form */
    int32_t flux;      /* face values: 0 MUSCL-minmod (Reading R2), 1 limited Lax-Wendroff */
    int32_t b_prev;    /* B of the recovery and of f_eq: 0 this step's (Reading R10), 1 the previous step's */
} orc_params;

/* ---------------------------------------------------------------- lattice */

typedef struct {
    double nu, ca, ct_c0, c0, ct; /* c_a = sqrt(19)/nu, c_t/c_0 = sqrt(27)/nu, c_0 = 3/8 (9 - 2 sqrt 3) */
    int e[Q19][3];                /* D3Q19 unit directions (Eq. cellconfigs1) */
    double w[Q19], wp[Q19];       /* weights of f and of g */
    double xi[Q19][4];            /* xi^mu_i = (c_t/c_0, c_a e_i) */
    double v[QH][3], ee[QH][3], bb[QH][3]; /* D3Q13 velocity, electric, magnetic vectors */
    int s[QH][3];                 /* lattice offset v dt / dx */
} orc_lattice;

/* D3Q19: rest, the 6 axis vectors, the 12 face diagonals (Eq. cellconfigs1).
 * The order is the interface order of the state arrays. */
static const int D3Q19[Q19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static void lattice_build(orc_lattice *L, double nu, double c, double dx, double dt)
{
    const double PI = 3.14159265358979323846;
    L->nu = nu;
    L->ca = sqrt(19.0) / nu;
    L->ct_c0 = sqrt(27.0) / nu;
    L->c0 = 3.0 / 8.0 * (9.0 - 2.0 * sqrt(3.0));
    L->ct = L->ct_c0 * L->c0;
    const double r2 = L->ct_c0 * L->ct_c0; /* c_t^2 / c_0^2 */
    const double ca2 = L->ca * L->ca;
    for (int i = 0; i < Q19; i++) {
        for (int a = 0; a < 3; a++) L->e[i][a] = D3Q19[i][a];
        /* weights of f: Sec. III, the three expressions below Eq. cellconfigs1 */
        if (i == 0)
            L->w[i] = 1.0 + 4.0 * r2 * nu * nu / 361.0 - r2 / ca2;
        else if (i <= 6)
            L->w[i] = r2 / (2166.0 * ca2) * (361.0 - 8.0 * ca2 * nu * nu);
        else
            L->w[i] = r2 * nu * nu / 1083.0;
        /* weights of g: the expressions below Eq. Hupp */
        if (i == 0)
            L->wp[i] = 0.1;
        else if (i <= 6)
            L->wp[i] = 0.3 - 1.0 / (6.0 * ca2);
        else
            L->wp[i] = 1.0 / (12.0 * ca2) - 3.0 / 40.0;
        L->xi[i][0] = L->ct_c0;
        for (int a = 0; a < 3; a++) L->xi[i][a + 1] = L->ca * L->e[i][a];
    }
    /* D3Q13 for the Maxwell equations (Sec. III, "Maxwell equations"):
     * v_i^p = 2c (cos, sin)((2i+1) pi / 4) in plane p (p=0: xy, p=1: xz, p=2: yz),
     * e_{i0} = v_{(i+3) mod 4} / 2, e_{i1} = v_{(i+1) mod 4} / 2, b_ij = v_i x e_ij / (2 c^2).
     * Population index k = 8 p + 2 i + j. */
    static const int plane_axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int p = 0; p < 3; p++) {
        double vp[4][3];
        for (int i = 0; i < 4; i++) {
            double th = (2 * i + 1) * PI / 4.0;
            for (int a = 0; a < 3; a++) vp[i][a] = 0.0;
            vp[i][plane_axes[p][0]] = 2.0 * c * cos(th);
            vp[i][plane_axes[p][1]] = 2.0 * c * sin(th);
        }
        for (int i = 0; i < 4; i++) {
            for (int j = 0; j < 2; j++) {
                int k = 8 * p + 2 * i + j;
                int other = (j == 0) ? (i + 3) % 4 : (i + 1) % 4;
                for (int a = 0; a < 3; a++) {
                    L->v[k][a] = vp[i][a];
                    L->ee[k][a] = 0.5 * vp[other][a];
                }
                const double *V = L->v[k], *Ev = L->ee[k];
                L->bb[k][0] = (V[1] * Ev[2] - V[2] * Ev[1]) / (2.0 * c * c);
                L->bb[k][1] = (V[2] * Ev[0] - V[0] * Ev[2]) / (2.0 * c * c);
                L->bb[k][2] = (V[0] * Ev[1] - V[1] * Ev[0]) / (2.0 * c * c);
                for (int a = 0; a < 3; a++) L->s[k][a] = (int)lround(L->v[k][a] * dt / dx);
            }
        }
    }
}

/* ---------------------------------------------------------------- context */

typedef struct {
    double eps, p, n, gam, beta[3], E[3], B[3], J[3], rhoc;
    double T[4][4], N0;
    double Tfl[4][4]; /* fluid tensor T - T_EM of the recovery */
    int fail, iters;
} orc_macro;

typedef struct {
    orc_params P;
    orc_lattice L;
    long N;
    double dt, eps0;
    double *f[2], *g[2], *hs[2], *Ep[2];
    double *Bp[2];    /* previous step's B (3 arrays of N) when b_prev = 1, else NULL */
    int cur;
    double *ftr, *gtr; /* transported f, g of the current step, [q*N + cell] */
    double *hpull;    /* pulled h of the current step, 25 per cell */
    orc_macro *mac;   /* macroscopic fields of the current step */
    long step;
    long n_failed;    /* failed recoveries in the last macroscopic pass */
    /* driven low-z face (Reading R23): two ghost planes below z = 0 of
     * post-collision f, g, h* and of E, fixed in time; [q][layer][y][x] */
    double *gf, *gg, *gh, *gE;
    double *Bt;       /* B of Eq. Cal_B from the streamed h of every cell, 3 arrays of N */
    double *Ez0;      /* initial E^z, for the reconnection rate */
    double *force;    /* external force density (3 arrays of N) or NULL (Reading R26) */
    double fgate;     /* the force acts while the previous step's max |beta| < fgate (<= 0: always) */
    double vmax;      /* max |beta| over the cells at the last step's recovery */
    double B0;        /* max |B| of the initial fields */
} orc_ctx;

static inline long cell_index(const orc_ctx *C, int x, int y, int z)
{
    return (long)x + (long)C->P.nx * ((long)y + (long)C->P.ny * (long)z);
}

/* Boundary mapping of one coordinate: periodic wrap, or for an open face the
 * ghost is a copy of the first interior cell along the face normal (Sec. IV,
 * Alfven test; Reading R19). */
static inline int map_coord(int x, int n, int lo, int hi)
{
    if (x < 0) {
        if (lo == BC_PERIODIC) return ((x % n) + n) % n;
        return 0; /* open; a driven face's ghost planes are read through value_at */
    }
    if (x >= n) {
        if (hi == BC_PERIODIC) return x % n;
        return n - 1;
    }
    return x;
}

static inline long nb_index(const orc_ctx *C, int x, int y, int z)
{
    const orc_params *P = &C->P;
    x = map_coord(x, P->nx, P->bc_lo[0], P->bc_hi[0]);
    y = map_coord(y, P->ny, P->bc_lo[1], P->bc_hi[1]);
    z = map_coord(z, P->nz, P->bc_lo[2], P->bc_hi[2]);
    return cell_index(C, x, y, z);
}

/* Reading R23: with a driven low-z face, z = -1 and z = -2 are ghost planes
 * whose post-collision populations and E are fixed (the equilibrium of the
 * prescribed face fields).  Value of array q of a distribution set at a
 * lattice point that may lie in a ghost plane: `arr` holds the interior
 * (nq arrays of N), `ghost` the two ghost planes of the same arrays. */
static inline int driven_ghost(const orc_ctx *C, int z)
{
    return C->P.bc_lo[2] == BC_DRIVEN && z < 0;
}

static inline double value_at(const orc_ctx *C, const double *arr, const double *ghost, int q, int x, int y, int z)
{
    const orc_params *P = &C->P;
    if (ghost && driven_ghost(C, z)) {
        int xx = map_coord(x, P->nx, P->bc_lo[0], P->bc_hi[0]);
        int yy = map_coord(y, P->ny, P->bc_lo[1], P->bc_hi[1]);
        int layer = -z - 1; /* z = -1 -> 0, z = -2 -> 1 */
        long plane = (long)P->nx * P->ny;
        return ghost[((long)q * 2 + layer) * plane + xx + (long)P->nx * yy];
    }
    return arr[(long)q * C->N + nb_index(C, x, y, z)];
}

/* ------------------------------------------------------------ physics bits */

/* Components of the electromagnetic energy-momentum tensor as listed in
 * Sec. III above Eq. Dis_fun_EM (Reading R8: these components, not the
 * covariant Eq. EM_EM, fix the sign). */
static void t_em(double eps0, double c, const double E[3], const double B[3], double T[4][4])
{
    double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double U = 0.5 * (E2 + c * c * B2);
    double ExB[3] = {E[1] * B[2] - E[2] * B[1], E[2] * B[0] - E[0] * B[2], E[0] * B[1] - E[1] * B[0]};
    T[0][0] = eps0 * U;
    for (int a = 0; a < 3; a++) {
        T[0][a + 1] = eps0 * c * ExB[a]; /* (1 / (mu0 c)) (E x B) with eps0 mu0 c^2 = 1 */
        T[a + 1][0] = T[0][a + 1];
        for (int b = 0; b < 3; b++)
            T[a + 1][b + 1] = eps0 * (-E[a] * E[b] - c * c * B[a] * B[b] + (a == b ? U : 0.0));
    }
}

/* Relativistic Ohm's law, Eq. Ohm. */
static void ohm_current(const orc_ctx *C, const double E[3], const double u[3], const double B[3], double rhoc,
                        double J[3])
{
    double c = C->P.c;
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double gam = 1.0 / sqrt(1.0 - u2 / (c * c));
    double uxB[3] = {u[1] * B[2] - u[2] * B[1], u[2] * B[0] - u[0] * B[2], u[0] * B[1] - u[1] * B[0]};
    double Eu = E[0] * u[0] + E[1] * u[1] + E[2] * u[2];
    for (int a = 0; a < 3; a++)
        J[a] = C->P.sigma * gam * (E[a] + uxB[a] - Eu * u[a] / (c * c)) + rhoc * u[a];
}

/* Gaussian elimination with partial pivoting for a 3x3 system. */
static void solve3(double A[3][3], double b[3], double x[3])
{
    for (int col = 0; col < 3; col++) {
        int piv = col;
        for (int r = col + 1; r < 3; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col) {
            for (int k = 0; k < 3; k++) {
                double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < 3; r++) {
            double m = A[r][col] / A[col][col];
            for (int k = col; k < 3; k++) A[r][k] -= m * A[col][k];
            b[r] -= m * b[col];
        }
    }
    for (int r = 2; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < 3; k++) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
}

/* E from E = E' - (dt/2) mu0 c^2 J(E) with J from Ohm's law (Eq. Ex_force):
 * (1+K) E - (K/c^2)(E.u) u = E' - K (u x B) - (dt/2) mu0 c^2 rho_c u,
 * K = (dt/2) mu0 c^2 sigma gamma, written as a 3x3 system and solved
 * directly.  Then J from Ohm's law. */
static void ohm_solve(const orc_ctx *C, const double Epr[3], const double B[3], const double u[3], double rhoc,
                      double E[3], double J[3])
{
    double c = C->P.c;
    double q = 0.5 * C->dt * C->P.mu0 * c * c;
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double gam = 1.0 / sqrt(1.0 - u2 / (c * c));
    double K = q * C->P.sigma * gam;
    double uxB[3] = {u[1] * B[2] - u[2] * B[1], u[2] * B[0] - u[0] * B[2], u[0] * B[1] - u[1] * B[0]};
    double A[3][3], rhs[3];
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) A[a][b] = (a == b ? 1.0 + K : 0.0) - K * u[a] * u[b] / (c * c);
        rhs[a] = Epr[a] - K * uxB[a] - q * rhoc * u[a];
    }
    solve3(A, rhs, E);
    ohm_current(C, E, u, B, rhoc, J);
}

/* Landau-frame recovery (Sec. III, "Coupling between fluid and
 * electromagnetic fields"): the four-velocity is the eigenvector of the
 * largest eigenvalue of the fluid tensor T_fl^mu_nu = T_fl^{mu lam} eta_{lam nu},
 * eta = diag(+,-,-,-), found by the power method.  Reading R8: the paper's
 * tensor T - eps0 F F equals T_fl + s eta with a scalar s, so it has the same
 * eigenvector and an eigenvalue shifted by s; the iteration runs on T_fl and
 * its eigenvalue is eps directly.  The eigenvector is normalised to
 * U^0 = 1, so its spatial part is beta = u / c. */
static int power_method(const double T[4][4], double beta[3], double *lam, int *iters)
{
    double x[4] = {1.0, 0.0, 0.0, 0.0};
    double prev = HUGE_VAL;
    int it;
    for (it = 1; it <= 5000; it++) {
        double y[4];
        for (int mu = 0; mu < 4; mu++) y[mu] = T[mu][0] * x[0] - T[mu][1] * x[1] - T[mu][2] * x[2] - T[mu][3] * x[3];
        if (!(y[0] > 0.0) || !isfinite(y[0])) {
            *iters = it;
            return -1;
        }
        double change = 0.0;
        for (int mu = 1; mu < 4; mu++) {
            double xn = y[mu] / y[0];
            double d = fabs(xn - x[mu]);
            if (d > change) change = d;
            x[mu] = xn;
        }
        if (change == 0.0) break;
        if (change >= prev && change < 1e-13) break; /* stagnated at rounding level */
        prev = change;
    }
    *iters = it;
    if (it > 5000) return -1;
    *lam = T[0][0] - T[0][1] * x[1] - T[0][2] * x[2] - T[0][3] * x[3];
    for (int a = 0; a < 3; a++) beta[a] = x[a + 1];
    return 0;
}

/* Equilibrium of f, Eq. Dis_fun_EM, in the paper's variables
 * chi^mu = U^mu / c_s = gamma nu (1, beta), c_i = c_a e_i.
 * Reading R7, four corrections to the printed equation, each forced by the
 * requirement that the moments of f_eq be T_fluid + T_EM:
 *  (1) the delta_{i0} coefficient is 361 (3p - eps) / (33 (p + eps)), which
 *      vanishes for eps = 3p as the text says; the printed one is -361/33;
 *  (2) the (nu^2/5)[c^2 (B.c_i)^2 + (E.c_i)^2] term enters with a minus sign;
 *  (3) the third cross term is c_i^y c_i^z E^y E^z (and the same for B);
 *  (4) the (B x E).c_i term carries a factor c (invisible at c = 1).
 * Reading R6: eps includes the rest mass, p = (Gamma-1)(eps - n c^2). */
static void f_equilibrium(const orc_ctx *C, double eps, double p, const double beta[3], const double E[3],
                          const double B[3], double feq[Q19])
{
    const orc_lattice *L = &C->L;
    const double nu = L->nu, c = C->P.c, eps0 = C->eps0;
    const double r = 1.0 / (L->ct_c0 * L->ct_c0); /* c_0^2 / c_t^2 */
    double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    double gam = 1.0 / sqrt(1.0 - b2);
    double chi0 = gam * nu;
    double chi[3] = {gam * nu * beta[0], gam * nu * beta[1], gam * nu * beta[2]};
    double chichi = chi[0] * chi[0] + chi[1] * chi[1] + chi[2] * chi[2];
    double A = (3.0 * p - eps) / (p + eps);
    double Bcoef = 361.0 * (3.0 * p - eps) / (33.0 * (p + eps));
    double first = L->ct * chi0 / (2.0 * L->c0 * L->c0) - chi0 / (nu * L->c0);
    double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double BxE[3] = {B[1] * E[2] - B[2] * E[1], B[2] * E[0] - B[0] * E[2], B[0] * E[1] - B[1] * E[0]};
    for (int i = 0; i < Q19; i++) {
        double ci[3];
        for (int a = 0; a < 3; a++) ci[a] = L->ca * L->e[i][a];
        double cchi = ci[0] * chi[0] + ci[1] * chi[1] + ci[2] * chi[2];
        double cross = ci[0] * ci[1] * chi[0] * chi[1] + ci[0] * ci[2] * chi[0] * chi[2] + ci[1] * ci[2] * chi[1] * chi[2];
        double diag = ci[0] * ci[0] * chi[0] * chi[0] + ci[1] * ci[1] * chi[1] * chi[1] + ci[2] * ci[2] * chi[2] * chi[2];
        double fluid = 1.0 + A + (i == 0 ? Bcoef : 0.0) + cross + first * cchi +
                       4.0 / 15.0 * (diag - 4.0 / (nu * nu) * chichi);
        double Bc = B[0] * ci[0] + B[1] * ci[1] + B[2] * ci[2];
        double Ec = E[0] * ci[0] + E[1] * ci[1] + E[2] * ci[2];
        double BxEc = BxE[0] * ci[0] + BxE[1] * ci[1] + BxE[2] * ci[2];
        double crossEB = ci[0] * ci[1] * (E[0] * E[1] + c * c * B[0] * B[1]) +
                         ci[0] * ci[2] * (E[0] * E[2] + c * c * B[0] * B[2]) +
                         ci[1] * ci[2] * (E[1] * E[2] + c * c * B[1] * B[2]);
        double em = 1.5 * (c * c * B2 + E2) + 0.8 * (c * c * B2 + E2) - nu / sqrt(3.0) * c * BxEc -
                    nu * nu / 5.0 * (c * c * Bc * Bc + Ec * Ec) - 7.0 * nu * nu / 20.0 * crossEB;
        feq[i] = 0.75 * (eps + p) * r * L->w[i] * fluid + r * eps0 * L->w[i] * em;
    }
}

/* Equilibrium of g, Eq. Hupp; Reading R12: the velocity in it is beta = u/c. */
static void g_equilibrium(const orc_ctx *C, double n, const double beta[3], double geq[Q19])
{
    const orc_lattice *L = &C->L;
    double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    double gam = 1.0 / sqrt(1.0 - b2);
    for (int i = 0; i < Q19; i++) {
        double cu = L->ca * (L->e[i][0] * beta[0] + L->e[i][1] * beta[1] + L->e[i][2] * beta[2]);
        geq[i] = L->wp[i] * n * gam * (1.0 / L->ct_c0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * b2);
    }
}

/* Equilibrium of h, Eq. Maxwell-eq.  Reading R13: the current coefficient is
 * 1/(32 c^2), so that sum_k h_eq v_k = J for every c; the printed 1/16 is that
 * value at c = 1/sqrt(2). */
static void h_equilibrium(const orc_ctx *C, const double J[3], const double E[3], const double B[3], double rhoc,
                          double heq[QH + 1])
{
    const orc_lattice *L = &C->L;
    double c = C->P.c;
    for (int k = 0; k < QH; k++) {
        double vJ = L->v[k][0] * J[0] + L->v[k][1] * J[1] + L->v[k][2] * J[2];
        double Ee = E[0] * L->ee[k][0] + E[1] * L->ee[k][1] + E[2] * L->ee[k][2];
        double Bb = B[0] * L->bb[k][0] + B[1] * L->bb[k][1] + B[2] * L->bb[k][2];
        heq[k] = vJ / (32.0 * c * c) + Ee / (8.0 * c * c) + Bb / 8.0;
    }
    heq[QH] = rhoc;
}

/* ------------------------------------------------------------ transport */

static inline double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* Reading R2: the face flux h_i^a of Eq. rlb (defined in a reference the
 * paper cites) is taken along the lattice link of population i: a MUSCL
 * reconstruction with a minmod-limited slope, upwinded along e_i, between the
 * lattice neighbours x - 2 e_i .. x + e_i.  The Courant number along the link
 * is (c_0/c_t) c_a c dt/dx = sqrt(19/54) for every moving population
 * (Reading R17: time enters as x^0 = c t).  For the six axis populations this
 * is the printed axis-wise difference; for the face diagonals the axis-wise
 * unsplit form has C_x + C_y = 1.19 > 1 and is unstable.  The alternative
 * reading (flux = 1) is the limited Lax-Wendroff face value, whose slope term
 * carries the factor (1 - C): exact translation of quadratic profiles.
 * Returns the flux difference (dt/dx)(c_0/c_t) [h(x + e_i/2) - h(x - e_i/2)]. */
static double advection(const orc_ctx *C, const double *arr, const double *ghost, int i, int x, int y, int z)
{
    const orc_lattice *L = &C->L;
    if (i == 0) return 0.0;
    const int *e = L->e[i];
    double cour = (1.0 / L->ct_c0) * L->ca * C->P.c * C->dt / C->P.dx;
    double fm2 = value_at(C, arr, ghost, i, x - 2 * e[0], y - 2 * e[1], z - 2 * e[2]);
    double fm1 = value_at(C, arr, ghost, i, x - e[0], y - e[1], z - e[2]);
    double f0 = value_at(C, arr, ghost, i, x, y, z);
    double fp1 = value_at(C, arr, ghost, i, x + e[0], y + e[1], z + e[2]);
    double s = C->P.flux == 1 ? 0.5 * (1.0 - cour) : 0.5;
    double face_plus = f0 + s * minmod(f0 - fm1, fp1 - f0);     /* face x + e_i/2, upwind cell x */
    double face_minus = fm1 + s * minmod(fm1 - fm2, f0 - fm1);  /* face x - e_i/2, upwind cell x - e_i */
    return cour * (face_plus - face_minus);
}

/* Reading R5: the bulk-viscosity term is lambda_i times the 7-point central
 * Laplacian of f_i itself. */
static double laplacian(const orc_ctx *C, const double *arr, const double *ghost, int i, int x, int y, int z)
{
    double c0 = value_at(C, arr, ghost, i, x, y, z);
    double s = 0.0;
    s += value_at(C, arr, ghost, i, x + 1, y, z) + value_at(C, arr, ghost, i, x - 1, y, z) - 2.0 * c0;
    s += value_at(C, arr, ghost, i, x, y + 1, z) + value_at(C, arr, ghost, i, x, y - 1, z) - 2.0 * c0;
    s += value_at(C, arr, ghost, i, x, y, z + 1) + value_at(C, arr, ghost, i, x, y, z - 1) - 2.0 * c0;
    return s;
}

/* ------------------------------------------------------------ macroscopic */

/* eps0 div E by central differences over the neighbours (boundary mapping
 * as for the distributions); E is stored as three arrays of N values, and
 * `ghost` holds E in the ghost planes of a driven face (NULL: none). */
static double gauss_charge(const orc_ctx *C, const double *E, const double *ghost, int x, int y, int z)
{
    double dv = (value_at(C, E, ghost, 0, x + 1, y, z) - value_at(C, E, ghost, 0, x - 1, y, z) +
                 value_at(C, E, ghost, 1, x, y + 1, z) - value_at(C, E, ghost, 1, x, y - 1, z) +
                 value_at(C, E, ghost, 2, x, y, z + 1) - value_at(C, E, ghost, 2, x, y, z - 1)) /
                (2.0 * C->P.dx);
    return C->eps0 * dv;
}

/* Derivative along `axis` of a field X (N values) at a cell: central
 * differences, periodic wrap on periodic axes; on the faces of a
 * non-periodic axis the one-sided difference towards the interior; zero on
 * an axis of one cell.  This is the divergence operator of the normal-B
 * adjustment and of the max |div B| diagnostic. */
static double axis_derivative(const orc_ctx *C, const double *X, int axis, int x, int y, int z)
{
    const orc_params *P = &C->P;
    const int n = axis == 0 ? P->nx : (axis == 1 ? P->ny : P->nz);
    const int v = axis == 0 ? x : (axis == 1 ? y : z);
    const int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    if (n == 1) return 0.0;
    const int periodic = P->bc_lo[axis] == BC_PERIODIC;
    const double here = X[cell_index(C, x, y, z)];
    if (!periodic && v == 0) return (X[cell_index(C, x + ex, y + ey, z + ez)] - here) / P->dx;
    if (!periodic && v == n - 1) return (here - X[cell_index(C, x - ex, y - ey, z - ez)]) / P->dx;
    return (X[nb_index(C, x + ex, y + ey, z + ez)] - X[nb_index(C, x - ex, y - ey, z - ez)]) / (2.0 * P->dx);
}

/* Reading R22 (the divergence-free adjustment on open faces, Sec. IV, KH
 * set-up): in a cell on an open face of axis a (with at least two cells
 * along a) and on no face of another non-periodic axis, the normal
 * component of B is replaced by the value that makes the discrete
 * divergence zero there, using the streamed B of the inner neighbour and the
 * tangential derivatives of the streamed B:
 *   low face:  B_a(x) = B_a(x + e_a) + dx sum_{b != a} d_b B_b
 *   high face: B_a(x) = B_a(x - e_a) - dx sum_{b != a} d_b B_b.
 * Every other component (and every interior, edge or corner cell) keeps the
 * streamed value.  The adjusted B is the cell's B in the fluid coupling
 * (recovery, Ohm's law, f_eq); the Maxwell populations relax towards h_eq of
 * the streamed B (see collision_pass).  Edge cells are left alone because
 * their two adjustments assume each other's unadjusted value; with them the
 * fields grew at the corners of a box open on every face.
 * Fills B with the cell's B for this step. */
static void divb_fixed_B(const orc_ctx *C, int x, int y, int z, double B[3])
{
    const orc_params *P = &C->P;
    const long N = C->N;
    const long id = cell_index(C, x, y, z);
    for (int a = 0; a < 3; a++) B[a] = C->Bt[(long)a * N + id];
    if (!P->divb_fix) return;
    const int dims[3] = {P->nx, P->ny, P->nz}, pos[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        const int n = dims[a];
        if (n < 2) continue;
        const int low = pos[a] == 0 && P->bc_lo[a] == BC_OPEN;
        const int high = pos[a] == n - 1 && P->bc_hi[a] == BC_OPEN;
        if (!low && !high) continue;
        int edge = 0;
        for (int b = 0; b < 3; b++)
            if (b != a && dims[b] >= 2 && P->bc_lo[b] != BC_PERIODIC && (pos[b] == 0 || pos[b] == dims[b] - 1))
                edge = 1;
        if (edge) continue;
        double dt_sum = 0.0;
        for (int b = 0; b < 3; b++)
            if (b != a) dt_sum += axis_derivative(C, C->Bt + (long)b * N, b, x, y, z);
        const int ex = a == 0, ey = a == 1, ez = a == 2;
        if (low)
            B[a] = C->Bt[(long)a * N + cell_index(C, x + ex, y + ey, z + ez)] + P->dx * dt_sum;
        else
            B[a] = C->Bt[(long)a * N + cell_index(C, x - ex, y - ey, z - ez)] - P->dx * dt_sum;
    }
}

/* The first half of one step at one cell: transport f and g, stream h, take
 * the moments, recover the fluid state with the previous step's E and B,
 * then B, E (with the current as a force) and J (Sec. III, coupling).
 *
 * Reading R4: the state between steps is post-collision.  Eq. rlb is applied
 * as collide-then-transport: the face fluxes and the bulk-viscosity term act
 * on the post-collision f, and the collision acts on the transported f with
 * the equilibrium of the transported moments.  (The unsplit forward-Euler
 * form amplifies the grid-scale non-equilibrium mode by 1 - omega - 2C, with
 * C = sqrt(19/54) the Courant number, so it is unstable at the paper's
 * tau = 1; the printed f(t + dt) in the collision is not conservative.) */
static void macroscopic_cell(orc_ctx *C, int x, int y, int z, orc_macro *m, const double *hp)
{
    const orc_lattice *L = &C->L;
    const orc_params *P = &C->P;
    const long N = C->N;
    const long id = cell_index(C, x, y, z);
    const double *fs = C->f[C->cur], *gs = C->g[C->cur];
    const double *Ep = C->Ep[C->cur];
    const double c = P->c;
    /* Reading R5: lambda_i = alpha dx for i != 0 times the 7-point Laplacian,
     * with time as c dt (coefficient alpha c dt / dx); the prefactor c_0 nu / c_t
     * of Eq. rlb is not applied to this term (at nu = sqrt(27) it would be
     * sqrt(27), and the explicit term would exceed the diffusion limit 1/6). */
    const double kv = P->alpha * P->dx * P->c * C->dt / (P->dx * P->dx);
    double *f = C->ftr, *g = C->gtr;

    /* transport (left-hand side and bulk-viscosity term of Eq. rlb) */
    for (int i = 0; i < Q19; i++) {
        double val = fs[(long)i * N + id] - advection(C, fs, C->gf, i, x, y, z);
        if (i != 0) val += kv * laplacian(C, fs, C->gf, i, x, y, z);
        f[(long)i * N + id] = val;
        g[(long)i * N + id] = gs[(long)i * N + id] - advection(C, gs, C->gg, i, x, y, z);
    }

    /* T^{mu nu} = sum_i xi^mu_i xi^nu_i f_i and N^0 = sum_i xi^0_i g_i */
    for (int mu = 0; mu < 4; mu++)
        for (int nv = 0; nv < 4; nv++) {
            double s = 0.0;
            for (int i = 0; i < Q19; i++) s += L->xi[i][mu] * L->xi[i][nv] * f[(long)i * N + id];
            m->T[mu][nv] = s;
        }
    double N0 = 0.0;
    for (int i = 0; i < Q19; i++) N0 += L->xi[i][0] * g[(long)i * N + id];
    m->N0 = N0;

    /* Eqs. Cal_E, Cal_rhoc from the streamed h; B of Eq. Cal_B was taken by
     * the streaming pass, with the normal component adjusted on open faces */
    double Epr[3] = {0, 0, 0}, B[3], rhoc = hp[QH];
    for (int k = 0; k < QH; k++) {
        for (int a = 0; a < 3; a++) Epr[a] += hp[k] * L->ee[k][a];
        rhoc += hp[k];
    }
    divb_fixed_B(C, x, y, z, B);

    /* Fluid tensor T_fl = T - T_EM.  Reading R10: E is the previous step's
     * (the current one needs the velocity through Ohm's law, Eq. Ex_force);
     * B is this step's, a moment of the streamed h (Eq. Cal_B) that does not
     * depend on the recovery.  The same pair enters f_eq below.  With
     * b_prev = 1, B is the previous step's as well, the paper's wording of
     * the coupling subsection (Sec. III). */
    double Eprev[3], Brec[3], Tem[4][4], Tfl[4][4];
    for (int a = 0; a < 3; a++) {
        Eprev[a] = Ep[(long)a * N + id];
        Brec[a] = P->b_prev ? C->Bp[C->cur][(long)a * N + id] : B[a];
    }
    t_em(C->eps0, c, Eprev, Brec, Tem);
    for (int mu = 0; mu < 4; mu++)
        for (int nv = 0; nv < 4; nv++) m->Tfl[mu][nv] = Tfl[mu][nv] = m->T[mu][nv] - Tem[mu][nv];

    double beta[3], lam = NAN;
    int it = 0;
    int bad = power_method(Tfl, beta, &lam, &it);
    m->iters = it;
    double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    double gam = 1.0 / sqrt(1.0 - b2);
    double n = N0 / gam; /* N^mu = n U^mu (Reading R11) */
    double p = (C->P.Gamma - 1.0) * (lam - n * c * c);
    if (bad || !(b2 < 1.0) || !(lam > 0.0) || !(n > 0.0) || !(p >= 0.0) || !isfinite(p)) {
        m->fail = 1;
        m->eps = m->p = m->n = m->gam = NAN;
        for (int a = 0; a < 3; a++) m->beta[a] = m->E[a] = m->J[a] = NAN;
        for (int a = 0; a < 3; a++) m->B[a] = B[a];
        m->rhoc = rhoc;
        return;
    }
    m->fail = 0;
    m->eps = lam;
    m->p = p;
    m->n = n;
    m->gam = gam;
    double u[3];
    for (int a = 0; a < 3; a++) {
        m->beta[a] = beta[a];
        u[a] = c * beta[a];
        m->B[a] = B[a];
    }
    m->rhoc = rhoc;
    /* Reading R20: the charge in the convection current rho_c u of Eq. Ohm is
     * Gauss's law (Eq. Gauss_E) applied to the previous step's E by central
     * differences.  With the populations' charge (Eq. Cal_rhoc) the
     * non-dissipative D3Q13 charge flux makes the convection current
     * unstable in any moving fluid. */
    double rho_gauss = gauss_charge(C, Ep, C->gE, x, y, z);
    ohm_solve(C, Epr, B, u, rho_gauss, m->E, m->J);
}

/* Stream h of every cell (Eq. LB_Maxwell: h_k(x, t) = h*_k(x - v_k dt, t - dt),
 * the rest population in place) and take B of Eq. Cal_B from it. */
static void stream_pass(orc_ctx *C)
{
    const orc_lattice *L = &C->L;
    const long N = C->N;
    const double *hs = C->hs[C->cur];
    for (int z = 0; z < C->P.nz; z++)
        for (int y = 0; y < C->P.ny; y++)
            for (int x = 0; x < C->P.nx; x++) {
                long id = cell_index(C, x, y, z);
                double *hp = &C->hpull[id * (QH + 1)];
                for (int k = 0; k < QH; k++)
                    hp[k] = value_at(C, hs, C->gh, k, x - L->s[k][0], y - L->s[k][1], z - L->s[k][2]);
                hp[QH] = hs[(long)QH * N + id];
                for (int a = 0; a < 3; a++) {
                    double b = 0.0;
                    for (int k = 0; k < QH; k++) b += hp[k] * L->bb[k][a];
                    C->Bt[(long)a * N + id] = b;
                }
            }
}

static void macroscopic_pass(orc_ctx *C)
{
    long nf = 0;
    stream_pass(C);
    for (int z = 0; z < C->P.nz; z++)
        for (int y = 0; y < C->P.ny; y++)
            for (int x = 0; x < C->P.nx; x++) {
                long id = cell_index(C, x, y, z);
                macroscopic_cell(C, x, y, z, &C->mac[id], &C->hpull[id * (QH + 1)]);
                nf += C->mac[id].fail;
            }
    C->n_failed = nf;
}

/* The second half of one step: equilibria (f_eq with the previous step's E
 * and this step's B, as in the recovery; h_eq with the new E, B), the collisions of f (Anderson-Witting, rate c_0 nu dt (xi_mu chi^mu /
 * nu^2) / (tau c_t)), g (rate c_0 nu dt / (tau c_t)) and h (Eq. LB_Maxwell),
 * and the carry of E, B to the next step. */
static void collision_pass(orc_ctx *C)
{
    const orc_lattice *L = &C->L;
    const orc_params *P = &C->P;
    const long N = C->N;
    const int dst = 1 - C->cur;
    const double *f = C->ftr, *g = C->gtr;
    double *fn = C->f[dst], *gn = C->g[dst], *hn = C->hs[dst], *En = C->Ep[dst];
    const double pref = L->nu / L->ct_c0; /* c_0 nu / c_t; dt / tau with tau in units of dt (Reading R3) */
    const double wg = pref / P->tau;

    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++)
            for (int x = 0; x < P->nx; x++) {
                long id = cell_index(C, x, y, z);
                const orc_macro *m = &C->mac[id];
                const double *hp = &C->hpull[id * (QH + 1)];
                double feq[Q19], geq[Q19], heq[QH + 1];
                /* Reading R10: f_eq carries T_EM of the same E, B pair that the
                 * recovery subtracted, so the collision conserves T^{0 nu} exactly */
                double Eprev[3], Brec[3];
                for (int a = 0; a < 3; a++) {
                    Eprev[a] = C->Ep[C->cur][(long)a * N + id];
                    Brec[a] = P->b_prev ? C->Bp[C->cur][(long)a * N + id] : m->B[a];
                }
                f_equilibrium(C, m->eps, m->p, m->beta, Eprev, Brec, feq);
                g_equilibrium(C, m->n, m->beta, geq);
                /* Reading R22: the Maxwell populations relax towards h_eq of the
                 * streamed B.  With tau_h = 1/2 the collision reflects h about h_eq,
                 * so an adjusted B in h_eq would enter the populations twice over
                 * each step; that feedback made open boxes unstable (measured). */
                double Bstream[3];
                for (int a = 0; a < 3; a++) Bstream[a] = C->Bt[(long)a * N + id];
                h_equilibrium(C, m->J, m->E, Bstream, m->rhoc, heq);
                /* chi^mu = gamma nu (1, beta) */
                double chi[4] = {m->gam * L->nu, m->gam * L->nu * m->beta[0], m->gam * L->nu * m->beta[1],
                                 m->gam * L->nu * m->beta[2]};
                for (int i = 0; i < Q19; i++) {
                    /* xi_mu chi^mu with eta = diag(+,-,-,-) */
                    double xichi = L->xi[i][0] * chi[0] - L->xi[i][1] * chi[1] - L->xi[i][2] * chi[2] -
                                   L->xi[i][3] * chi[3];
                    double om = pref * (xichi / (L->nu * L->nu)) / P->tau;
                    /* Reading R4: explicit in f; with rates proportional to xi_mu chi^mu
                     * and the Landau-frame eigenpair this conserves T^{0 nu} exactly.
                     * Optionally (collision = 1) Eq. rlb as printed, with f(x, t + dt)
                     * in the collision term, in closed form: f' = (f + om f_eq) / (1 + om);
                     * the direction-dependent rate makes it only approximately conservative */
                    double fi = f[(long)i * N + id];
                    if (P->collision == 1)
                        fn[(long)i * N + id] = (fi + om * feq[i]) / (1.0 + om);
                    else
                        fn[(long)i * N + id] = fi - om * (fi - feq[i]);
                    /* Eq. rlb with g(x, t + dt) in the collision, in closed form; the rate
                     * is the same for every direction, so sum_i g is conserved */
                    double gi = g[(long)i * N + id];
                    gn[(long)i * N + id] = (gi + wg * geq[i]) / (1.0 + wg);
                }
                for (int k = 0; k <= QH; k++) hn[(long)k * N + id] = hp[k] - (hp[k] - heq[k]) / P->tau_h;
                for (int a = 0; a < 3; a++) En[(long)a * N + id] = m->E[a];
                /* b_prev = 1: this step's B (as the fluid coupling used it) is the next one's previous B */
                if (P->b_prev)
                    for (int a = 0; a < 3; a++) C->Bp[dst][(long)a * N + id] = m->B[a];
            }
    /* Reading R26: an external force density F (the flare's driver, Sec. IV) enters
     * as a source after the collision: c dt F^a into T^{0a} through the moving
     * populations, (19/9) w_i (e_i . c dt F) / kappa (sum_i w_i e_i^a e_i^b =
     * (9/19) delta^ab, no change of T^00 or T^ab), and the work c dt F . beta into
     * T^00 through the rest population.  It acts while the largest |beta| of the
     * previous step's recovery is below the gate (one-step lag). */
    double vmax = 0.0;
    for (long id = 0; id < N; id++) {
        const orc_macro *m = &C->mac[id];
        const double b = sqrt(m->beta[0] * m->beta[0] + m->beta[1] * m->beta[1] + m->beta[2] * m->beta[2]);
        if (b > vmax) vmax = b;
    }
    if (C->force && (C->fgate <= 0.0 || C->vmax < C->fgate)) {
        const double kap = sqrt(19.0 / 27.0), cdt = P->c * C->dt;
        for (long id = 0; id < N; id++) {
            const orc_macro *m = &C->mac[id];
            double F[3];
            for (int a = 0; a < 3; a++) F[a] = cdt * C->force[(long)a * N + id];
            fn[id] += F[0] * m->beta[0] + F[1] * m->beta[1] + F[2] * m->beta[2];
            for (int i = 1; i < Q19; i++) {
                const double eF = L->e[i][0] * F[0] + L->e[i][1] * F[1] + L->e[i][2] * F[2];
                fn[(long)i * N + id] += (19.0 / 9.0) * L->w[i] * eF / kap;
            }
        }
    }
    C->vmax = vmax;
    C->cur = dst;
    C->step++;
}

/* ------------------------------------------------------------ public API */

#define ORC_API __attribute__((visibility("default")))

ORC_API int rmhdlb_oracle_create(const orc_params *P, void **out)
{
    if (!P || !out) return ORC_EINVAL;
    *out = NULL;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return ORC_EINVAL;
    if (!(P->dx > 0) || !(P->c > 0) || !(P->mu0 > 0) || !(P->tau > 0) || !(P->Gamma > 1) || !(P->sigma >= 0) ||
        !(P->nu > 0) || !(P->alpha >= 0))
        return ORC_EINVAL;
    for (int a = 0; a < 3; a++) {
        int lo_ok = P->bc_lo[a] == BC_PERIODIC || P->bc_lo[a] == BC_OPEN || (a == 2 && P->bc_lo[a] == BC_DRIVEN);
        if (!lo_ok || (P->bc_hi[a] != BC_PERIODIC && P->bc_hi[a] != BC_OPEN)) return ORC_EINVAL;
        if ((P->bc_lo[a] == BC_PERIODIC) != (P->bc_hi[a] == BC_PERIODIC)) return ORC_EINVAL;
    }
    if (P->divb_fix != 0 && P->divb_fix != 1) return ORC_EINVAL;
    if (P->collision != 0 && P->collision != 1) return ORC_EINVAL;
    if (P->flux != 0 && P->flux != 1) return ORC_EINVAL;
    if (P->b_prev != 0 && P->b_prev != 1) return ORC_EINVAL;
    if (P->tau_h != 0.5) return ORC_EUNSUPPORTED; /* Eq. Ex_force holds for tau_h = 1/2 */
    orc_ctx *C = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!C) return ORC_ENOMEM;
    C->P = *P;
    C->N = (long)P->nx * P->ny * P->nz;
    C->dt = P->dx / (sqrt(2.0) * P->c); /* dx/dt = sqrt(2) c */
    C->eps0 = 1.0 / (P->mu0 * P->c * P->c);
    lattice_build(&C->L, P->nu, P->c, P->dx, C->dt);
    for (int b = 0; b < 2; b++) {
        C->f[b] = (double *)calloc((size_t)Q19 * C->N, sizeof(double));
        C->g[b] = (double *)calloc((size_t)Q19 * C->N, sizeof(double));
        C->hs[b] = (double *)calloc((size_t)(QH + 1) * C->N, sizeof(double));
        C->Ep[b] = (double *)calloc((size_t)3 * C->N, sizeof(double));
        if (P->b_prev) C->Bp[b] = (double *)calloc((size_t)3 * C->N, sizeof(double));
    }
    C->ftr = (double *)calloc((size_t)Q19 * C->N, sizeof(double));
    C->gtr = (double *)calloc((size_t)Q19 * C->N, sizeof(double));
    C->hpull = (double *)calloc((size_t)(QH + 1) * C->N, sizeof(double));
    C->mac = (orc_macro *)calloc((size_t)C->N, sizeof(orc_macro));
    C->Bt = (double *)calloc((size_t)3 * C->N, sizeof(double));
    C->Ez0 = (double *)calloc((size_t)C->N, sizeof(double));
    int ok = C->hpull && C->mac && C->ftr && C->gtr && C->Bt && C->Ez0;
    if (P->bc_lo[2] == BC_DRIVEN) {
        const size_t plane2 = (size_t)2 * P->nx * P->ny;
        C->gf = (double *)calloc(Q19 * plane2, sizeof(double));
        C->gg = (double *)calloc(Q19 * plane2, sizeof(double));
        C->gh = (double *)calloc((QH + 1) * plane2, sizeof(double));
        C->gE = (double *)calloc(3 * plane2, sizeof(double));
        ok = ok && C->gf && C->gg && C->gh && C->gE;
    }
    for (int b = 0; b < 2; b++) ok = ok && C->f[b] && C->g[b] && C->hs[b] && C->Ep[b] && (!P->b_prev || C->Bp[b]);
    if (!ok) {
        for (int b = 0; b < 2; b++) {
            free(C->f[b]);
            free(C->g[b]);
            free(C->hs[b]);
            free(C->Ep[b]);
            free(C->Bp[b]);
        }
        free(C->ftr);
        free(C->gtr);
        free(C->hpull);
        free(C->mac);
        free(C->Bt);
        free(C->Ez0);
        free(C->force);
        free(C->gf);
        free(C->gg);
        free(C->gh);
        free(C->gE);
        free(C);
        return ORC_ENOMEM;
    }
    *out = C;
    return ORC_OK;
}

ORC_API void rmhdlb_oracle_destroy(void *ctx)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C) return;
    for (int b = 0; b < 2; b++) {
        free(C->f[b]);
        free(C->g[b]);
        free(C->hs[b]);
        free(C->Ep[b]);
        free(C->Bp[b]);
    }
    free(C->ftr);
    free(C->gtr);
    free(C->hpull);
    free(C->mac);
    free(C->Bt);
    free(C->Ez0);
    free(C->force);
    free(C->gf);
    free(C->gg);
    free(C->gh);
    free(C->gE);
    free(C);
}

/* Reading R23: the ghost planes of a driven low-z face hold the
 * post-collision state of a fully relaxed cell with the prescribed fields:
 * f_eq and g_eq of (n, p, u, E = -u x B, B), h* = h_eq of (J, E + (dt/2)
 * mu0 c^2 J, B) with J of Eq. Ohm at zero charge (h* = h_eq is the fixed
 * point of the tau_h = 1/2 collision), and E.  Both ghost planes take the
 * same values; arrays are nx*ny values of the face, x fastest.  Returns
 * ORC_EINVAL for |u| >= c, n <= 0 or p < 0. */
static int fill_ghosts(orc_ctx *C, const double *n, const double *p, const double *const u[3],
                       const double *const B[3])
{
    const orc_params *P = &C->P;
    const long plane = (long)P->nx * P->ny;
    const double c = P->c;
    const double q = 0.5 * C->dt * P->mu0 * c * c;
    for (long xy = 0; xy < plane; xy++) {
        double uu[3] = {u[0][xy], u[1][xy], u[2][xy]}, BB[3] = {B[0][xy], B[1][xy], B[2][xy]};
        double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
        if (!(u2 < c * c) || !(n[xy] > 0) || !(p[xy] >= 0)) return ORC_EINVAL;
        double EE[3] = {-(uu[1] * BB[2] - uu[2] * BB[1]), -(uu[2] * BB[0] - uu[0] * BB[2]),
                        -(uu[0] * BB[1] - uu[1] * BB[0])};
        double beta[3] = {uu[0] / c, uu[1] / c, uu[2] / c};
        double eps = n[xy] * c * c + p[xy] / (P->Gamma - 1.0);
        double feq[Q19], geq[Q19], heq[QH + 1], JJ[3], Epr[3];
        f_equilibrium(C, eps, p[xy], beta, EE, BB, feq);
        g_equilibrium(C, n[xy], beta, geq);
        ohm_current(C, EE, uu, BB, 0.0, JJ);
        for (int a = 0; a < 3; a++) Epr[a] = EE[a] + q * JJ[a];
        h_equilibrium(C, JJ, Epr, BB, 0.0, heq);
        for (int layer = 0; layer < 2; layer++) {
            for (int i = 0; i < Q19; i++) {
                C->gf[((long)i * 2 + layer) * plane + xy] = feq[i];
                C->gg[((long)i * 2 + layer) * plane + xy] = geq[i];
            }
            for (int k = 0; k <= QH; k++) C->gh[((long)k * 2 + layer) * plane + xy] = heq[k];
            for (int a = 0; a < 3; a++) C->gE[((long)a * 2 + layer) * plane + xy] = EE[a];
        }
    }
    return ORC_OK;
}

/* Prescribed fields of a driven low-z face (Reading R23): n, p, u[3], B[3],
 * each nx*ny values.  Replaces the ghost planes set by rmhdlb_oracle_init. */
ORC_API int rmhdlb_oracle_set_driven(void *ctx, const double *n, const double *p, const double *const u[3],
                                     const double *const B[3])
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !n || !p || C->P.bc_lo[2] != BC_DRIVEN) return ORC_EINVAL;
    for (int a = 0; a < 3; a++)
        if (!u[a] || !B[a]) return ORC_EINVAL;
    return fill_ghosts(C, n, p, u, B);
}

/* Initial state from primitive fields, each an array of nx*ny*nz doubles in
 * x-fastest order: n, p, u (3 arrays), E, B, rho_c (NULL => eps0 div E by
 * central differences, Gauss's law as in the Alfven test).
 * The stored state is post-collision (Reading R4); the initial one is that of
 * a fully relaxed previous step, f* = f_eq and g* = g_eq of the given state,
 * and the previous-step E is the given E.  Reading R18: h* is laid out so that the first pull delivers
 * h_k = h_eq-form(J0, E'0, B0) with E'0 = E0 + (dt/2) mu0 c^2 J0, so the first
 * force-corrected E equals E0; h*_0 = rho_c. */
/* External force density (Reading R26): three arrays of N values in cell
 * order, copied; NULL switches the force off.  gate: the force acts while the
 * previous step's largest |beta| is below it (<= 0: always). */
ORC_API int rmhdlb_oracle_set_force(void *ctx, const double *const F[3], double gate)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C) return ORC_EINVAL;
    if (!F) {
        free(C->force);
        C->force = NULL;
        return ORC_OK;
    }
    for (int a = 0; a < 3; a++)
        if (!F[a]) return ORC_EINVAL;
    if (!C->force) C->force = (double *)malloc(sizeof(double) * 3 * (size_t)C->N);
    if (!C->force) return ORC_ENOMEM;
    for (int a = 0; a < 3; a++) memcpy(C->force + (long)a * C->N, F[a], sizeof(double) * (size_t)C->N);
    C->fgate = gate;
    return ORC_OK;
}

ORC_API int rmhdlb_oracle_init(void *ctx, const double *n, const double *p, const double *const u[3],
                               const double *const E[3], const double *const B[3], const double *rhoc_in)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !n || !p) return ORC_EINVAL;
    const long N = C->N;
    const orc_params *P = &C->P;
    const orc_lattice *L = &C->L;
    const double c = P->c;
    double *rhoc = (double *)malloc(sizeof(double) * N);
    double *J = (double *)malloc(sizeof(double) * 3 * N);
    if (!rhoc || !J) {
        free(rhoc);
        free(J);
        return ORC_ENOMEM;
    }
    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++)
            for (int x = 0; x < P->nx; x++) {
                long id = cell_index(C, x, y, z);
                if (rhoc_in) {
                    rhoc[id] = rhoc_in[id];
                } else {
                    double dv = (E[0][nb_index(C, x + 1, y, z)] - E[0][nb_index(C, x - 1, y, z)] +
                                 E[1][nb_index(C, x, y + 1, z)] - E[1][nb_index(C, x, y - 1, z)] +
                                 E[2][nb_index(C, x, y, z + 1)] - E[2][nb_index(C, x, y, z - 1)]) /
                                (2.0 * P->dx);
                    rhoc[id] = C->eps0 * dv;
                }
            }
    /* J0 from Ohm's law with the Gauss charge of E0 (Reading R20) */
    double *E0 = (double *)malloc(sizeof(double) * 3 * N);
    if (!E0) {
        free(rhoc);
        free(J);
        return ORC_ENOMEM;
    }
    for (int a = 0; a < 3; a++) memcpy(E0 + (long)a * N, E[a], sizeof(double) * N);
    int bad = 0;
    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++)
            for (int x = 0; x < P->nx; x++) {
                long id = cell_index(C, x, y, z);
                double uu[3] = {u[0][id], u[1][id], u[2][id]};
                double EE[3] = {E[0][id], E[1][id], E[2][id]}, BB[3] = {B[0][id], B[1][id], B[2][id]};
                double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
                if (!(u2 < c * c) || !(n[id] > 0) || !(p[id] >= 0)) bad = 1;
                double JJ[3];
                ohm_current(C, EE, uu, BB, gauss_charge(C, E0, NULL, x, y, z), JJ);
                for (int a = 0; a < 3; a++) J[(long)a * N + id] = JJ[a];
            }
    free(E0);
    if (bad) {
        free(rhoc);
        free(J);
        return ORC_EINVAL;
    }
    const int cur = C->cur;
    double *f = C->f[cur], *g = C->g[cur], *hs = C->hs[cur], *Ep = C->Ep[cur];
    const double q = 0.5 * C->dt * P->mu0 * c * c;
    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++)
            for (int x = 0; x < P->nx; x++) {
                long id = cell_index(C, x, y, z);
                double beta[3] = {u[0][id] / c, u[1][id] / c, u[2][id] / c};
                double EE[3] = {E[0][id], E[1][id], E[2][id]}, BB[3] = {B[0][id], B[1][id], B[2][id]};
                double eps = n[id] * c * c + p[id] / (P->Gamma - 1.0);
                double feq[Q19], geq[Q19];
                f_equilibrium(C, eps, p[id], beta, EE, BB, feq);
                g_equilibrium(C, n[id], beta, geq);
                for (int i = 0; i < Q19; i++) {
                    f[(long)i * N + id] = feq[i];
                    g[(long)i * N + id] = geq[i];
                }
                for (int k = 0; k < QH; k++) {
                    long t = nb_index(C, x + L->s[k][0], y + L->s[k][1], z + L->s[k][2]);
                    double Jt[3], Et[3], Bt[3], heq[QH + 1];
                    for (int a = 0; a < 3; a++) {
                        Jt[a] = J[(long)a * N + t];
                        Et[a] = E[a][t] + q * Jt[a];
                        Bt[a] = B[a][t];
                    }
                    h_equilibrium(C, Jt, Et, Bt, rhoc[t], heq);
                    hs[(long)k * N + id] = heq[k];
                }
                hs[(long)QH * N + id] = rhoc[id];
                for (int a = 0; a < 3; a++) Ep[(long)a * N + id] = EE[a];
                if (P->b_prev)
                    for (int a = 0; a < 3; a++) C->Bp[cur][(long)a * N + id] = BB[a];
            }
    free(rhoc);
    free(J);
    /* reference values of the reconnection-rate diagnostic */
    double b2max = 0.0;
    for (long id = 0; id < N; id++) {
        C->Ez0[id] = E[2][id];
        double b2 = fma(B[0][id], B[0][id], fma(B[1][id], B[1][id], B[2][id] * B[2][id]));
        if (b2 > b2max) b2max = b2;
    }
    C->B0 = sqrt(b2max);
    /* a driven face starts from the fields of its first interior plane */
    if (P->bc_lo[2] == BC_DRIVEN && fill_ghosts(C, n, p, u, B) != ORC_OK) return ORC_EINVAL;
    C->step = 0;
    C->vmax = 0.0;  /* the force gate starts open */
    return ORC_OK;
}

/* Advance nsteps time steps (transport and macroscopic pass, then collision). */
ORC_API int rmhdlb_oracle_step(void *ctx, long nsteps)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || nsteps < 0) return ORC_EINVAL;
    long failed = 0;
    for (long s = 0; s < nsteps; s++) {
        macroscopic_pass(C);
        failed += C->n_failed;
        collision_pass(C);
    }
    return failed ? ORC_ERECOVERY : ORC_OK;
}

/* Primitive fields of the current state (what the next step would compute
 * first).  Any output pointer may be NULL.  out order: n, p, eps, u[3], E[3],
 * B[3], J[3], rho_c; each nx*ny*nz doubles. */
ORC_API int rmhdlb_oracle_moments(void *ctx, double *const out[16], long *n_failed)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C) return ORC_EINVAL;
    macroscopic_pass(C);
    for (long id = 0; id < C->N; id++) {
        const orc_macro *m = &C->mac[id];
        double vals[16] = {m->n, m->p, m->eps, C->P.c * m->beta[0], C->P.c * m->beta[1], C->P.c * m->beta[2],
                           m->E[0], m->E[1], m->E[2], m->B[0], m->B[1], m->B[2], m->J[0], m->J[1], m->J[2],
                           m->rhoc};
        for (int q = 0; q < 16; q++)
            if (out[q]) out[q][id] = vals[q];
    }
    if (n_failed) *n_failed = C->n_failed;
    return C->n_failed ? ORC_ERECOVERY : ORC_OK;
}

/* Fluid tensor of the recovery of every cell of the current state and its
 * N^0: out[11 * cell + j] = T_fl^00, T_fl^0x, T_fl^0y, T_fl^0z, T_fl^xx,
 * T_fl^yy, T_fl^zz, T_fl^xy, T_fl^xz, T_fl^yz, N^0 (the inputs of the
 * learned recovery guess), and the recovered eps, beta in rec[4 * cell + j]. */
ORC_API int rmhdlb_oracle_fluid_tensor(void *ctx, double *out, double *rec)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !out) return ORC_EINVAL;
    macroscopic_pass(C);
    for (long id = 0; id < C->N; id++) {
        const orc_macro *m = &C->mac[id];
        double *o = out + 11 * id;
        o[0] = m->Tfl[0][0];
        o[1] = m->Tfl[0][1];
        o[2] = m->Tfl[0][2];
        o[3] = m->Tfl[0][3];
        o[4] = m->Tfl[1][1];
        o[5] = m->Tfl[2][2];
        o[6] = m->Tfl[3][3];
        o[7] = m->Tfl[1][2];
        o[8] = m->Tfl[1][3];
        o[9] = m->Tfl[2][3];
        o[10] = m->N0;
        if (rec) {
            rec[4 * id] = m->eps;
            for (int a = 0; a < 3; a++) rec[4 * id + 1 + a] = m->beta[a];
        }
    }
    return C->n_failed ? ORC_ERECOVERY : ORC_OK;
}

/* Charge density of the current state (h_0 + sum h, Eq. Cal_rhoc). */
ORC_API int rmhdlb_oracle_charge(void *ctx, double *rhoc)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !rhoc) return ORC_EINVAL;
    macroscopic_pass(C);
    for (long id = 0; id < C->N; id++) rhoc[id] = C->mac[id].rhoc;
    return ORC_OK;
}

/* Global diagnostics of the current state, sums in long double:
 * d[0] = sum T^00, d[1] = sum N^0, d[2..4] = sum T^0a, d[5] = sum eps0 (E^2 + c^2 B^2)/2,
 * d[6] = max |div B| (the derivative operator of axis_derivative), d[7] = sum rho_c,
 * d[8] = failed cells, d[9] = mean power-method iterations,
 * d[10] = reconnection rate, d[11] = null-point cell index, d[12] = B0.
 *
 * Reconnection rate (Sec. IV, KH reconnection; Reading R21): the null point
 * is the cell of least B_x^2 + B_y^2 (evaluated as fma(B_x, B_x, B_y B_y))
 * among the rows whose centre lies within null_band cells of y = 0, first in
 * x-fastest order on ties; R = (E^z - E^z_0) / B0 there, with E^z_0 the
 * initial E^z of that cell and B0 the largest |B| of the initial fields. */
ORC_API int rmhdlb_oracle_diagnostics(void *ctx, double d[13])
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !d) return ORC_EINVAL;
    macroscopic_pass(C);
    long double s[8] = {0};
    double maxdiv = 0.0;
    long double its = 0;
    const orc_params *P = &C->P;
    const long N = C->N;
    const double c = P->c;
    double *Bm = (double *)malloc(sizeof(double) * 3 * N);
    if (!Bm) return ORC_ENOMEM;
    for (long id = 0; id < N; id++)
        for (int a = 0; a < 3; a++) Bm[(long)a * N + id] = C->mac[id].B[a];
    const int band = P->null_band >= 1 ? P->null_band : 64;
    double best = INFINITY;
    long null_id = -1;
    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++)
            for (int x = 0; x < P->nx; x++) {
                long id = cell_index(C, x, y, z);
                const orc_macro *m = &C->mac[id];
                s[0] += m->T[0][0];
                s[1] += m->N0;
                for (int a = 0; a < 3; a++) s[2 + a] += m->T[0][a + 1];
                double E2 = m->E[0] * m->E[0] + m->E[1] * m->E[1] + m->E[2] * m->E[2];
                double B2 = m->B[0] * m->B[0] + m->B[1] * m->B[1] + m->B[2] * m->B[2];
                s[5] += 0.5 * C->eps0 * (E2 + c * c * B2);
                s[6] += m->rhoc;
                its += m->iters;
                double dv = 0.0;
                for (int a = 0; a < 3; a++) dv += axis_derivative(C, Bm + (long)a * N, a, x, y, z);
                if (fabs(dv) > maxdiv) maxdiv = fabs(dv);
                /* |y_j| <= band with cell centres y_j = j + 1/2 - ny/2 */
                if (labs(2L * y + 1 - P->ny) <= 2L * band) {
                    double key = fma(m->B[0], m->B[0], m->B[1] * m->B[1]);
                    if (key < best) {
                        best = key;
                        null_id = id;
                    }
                }
            }
    free(Bm);
    for (int k = 0; k < 6; k++) d[k] = (double)s[k];
    d[6] = maxdiv;
    d[7] = (double)s[6];
    d[8] = (double)C->n_failed;
    d[9] = (double)(its / (long double)N);
    d[10] = null_id >= 0 ? (C->mac[null_id].E[2] - C->Ez0[null_id]) / C->B0 : NAN;
    d[11] = (double)null_id;
    d[12] = C->B0;
    return ORC_OK;
}

/* Raw (post-collision) state in normalised variables F = (c_t/c_0)^2 f,
 * G = (c_t/c_0) g, in the order F[19], G[19], h*[25], E_prev[3] (then
 * B_prev[3] when b_prev = 1), each nx*ny*nz doubles. */
ORC_API int rmhdlb_oracle_get_state(void *ctx, double *out)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !out) return ORC_EINVAL;
    const long N = C->N;
    const double r2 = C->L.ct_c0 * C->L.ct_c0, r1 = C->L.ct_c0;
    const int b = C->cur;
    long o = 0;
    for (long k = 0; k < Q19 * N; k++) out[o++] = r2 * C->f[b][k];
    for (long k = 0; k < Q19 * N; k++) out[o++] = r1 * C->g[b][k];
    for (long k = 0; k < (QH + 1) * N; k++) out[o++] = C->hs[b][k];
    for (long k = 0; k < 3 * N; k++) out[o++] = C->Ep[b][k];
    if (C->P.b_prev)
        for (long k = 0; k < 3 * N; k++) out[o++] = C->Bp[b][k];
    return ORC_OK;
}

ORC_API int rmhdlb_oracle_set_state(void *ctx, const double *in)
{
    orc_ctx *C = (orc_ctx *)ctx;
    if (!C || !in) return ORC_EINVAL;
    const long N = C->N;
    const double r2 = C->L.ct_c0 * C->L.ct_c0, r1 = C->L.ct_c0;
    const int b = C->cur;
    long o = 0;
    for (long k = 0; k < Q19 * N; k++) C->f[b][k] = in[o++] / r2;
    for (long k = 0; k < Q19 * N; k++) C->g[b][k] = in[o++] / r1;
    for (long k = 0; k < (QH + 1) * N; k++) C->hs[b][k] = in[o++];
    for (long k = 0; k < 3 * N; k++) C->Ep[b][k] = in[o++];
    if (C->P.b_prev)
        for (long k = 0; k < 3 * N; k++) C->Bp[b][k] = in[o++];
    return ORC_OK;
}

ORC_API long rmhdlb_oracle_state_len(void *ctx)
{
    orc_ctx *C = (orc_ctx *)ctx;
    return C ? (long)(NSTATE + (C->P.b_prev ? 3 : 0)) * C->N : -1;
}

/* ---- single-cell entry points, used by the tests that pin the oracle ---- */

/* Lattice tables: e[19*3], w[19], wp[19], xi[19*4], v[24*3], ee[24*3], bb[24*3], s[24*3]. */
ORC_API int rmhdlb_oracle_lattice(const orc_params *P, int *e, double *w, double *wp, double *xi, double *v,
                                  double *ee, double *bb, int *s)
{
    if (!P) return ORC_EINVAL;
    orc_lattice L;
    double dt = P->dx / (sqrt(2.0) * P->c);
    lattice_build(&L, P->nu, P->c, P->dx, dt);
    for (int i = 0; i < Q19; i++) {
        for (int a = 0; a < 3; a++) e[3 * i + a] = L.e[i][a];
        w[i] = L.w[i];
        wp[i] = L.wp[i];
        for (int mu = 0; mu < 4; mu++) xi[4 * i + mu] = L.xi[i][mu];
    }
    for (int k = 0; k < QH; k++)
        for (int a = 0; a < 3; a++) {
            v[3 * k + a] = L.v[k][a];
            ee[3 * k + a] = L.ee[k][a];
            bb[3 * k + a] = L.bb[k][a];
            s[3 * k + a] = L.s[k][a];
        }
    return ORC_OK;
}

static int cell_ctx(const orc_params *P, orc_ctx *C)
{
    memset(C, 0, sizeof(*C));
    C->P = *P;
    C->dt = P->dx / (sqrt(2.0) * P->c);
    C->eps0 = 1.0 / (P->mu0 * P->c * P->c);
    lattice_build(&C->L, P->nu, P->c, P->dx, C->dt);
    return 0;
}

/* f_eq (paper variables, 19 values) and g_eq of one state. */
ORC_API int rmhdlb_oracle_equilibria(const orc_params *P, double eps, double p, double n, const double beta[3],
                                     const double E[3], const double B[3], double *feq, double *geq)
{
    orc_ctx C;
    cell_ctx(P, &C);
    if (feq) f_equilibrium(&C, eps, p, beta, E, B, feq);
    if (geq) g_equilibrium(&C, n, beta, geq);
    return ORC_OK;
}

/* h_eq of one state: 24 moving populations then the rest one. */
ORC_API int rmhdlb_oracle_h_equilibrium(const orc_params *P, const double J[3], const double E[3], const double B[3],
                                        double rhoc, double *heq)
{
    orc_ctx C;
    cell_ctx(P, &C);
    h_equilibrium(&C, J, E, B, rhoc, heq);
    return ORC_OK;
}

/* Recovery of one cell from T^{mu nu} (16 values, row-major), N^0 and the
 * previous step's E, B.  out: eps, p, n, beta[3]; returns iterations or <0. */
ORC_API int rmhdlb_oracle_recover(const orc_params *P, const double *T16, double N0, const double Eprev[3],
                                  const double Bprev[3], double *out)
{
    orc_ctx C;
    cell_ctx(P, &C);
    double Tem[4][4], Tfl[4][4];
    t_em(C.eps0, P->c, Eprev, Bprev, Tem);
    for (int mu = 0; mu < 4; mu++)
        for (int nv = 0; nv < 4; nv++) Tfl[mu][nv] = T16[4 * mu + nv] - Tem[mu][nv];
    double beta[3], lam;
    int it;
    if (power_method(Tfl, beta, &lam, &it)) return ORC_ERECOVERY;
    double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    double gam = 1.0 / sqrt(1.0 - b2);
    double n = N0 / gam;
    out[0] = lam;
    out[1] = (P->Gamma - 1.0) * (lam - n * P->c * P->c);
    out[2] = n;
    for (int a = 0; a < 3; a++) out[3 + a] = beta[a];
    return it;
}

/* E and J of one cell from E', B, u, rho_c (Eq. Ex_force with Eq. Ohm). */
ORC_API int rmhdlb_oracle_ohm(const orc_params *P, const double Epr[3], const double B[3], const double u[3],
                              double rhoc, double E[3], double J[3])
{
    orc_ctx C;
    cell_ctx(P, &C);
    ohm_solve(&C, Epr, B, u, rhoc, E, J);
    return ORC_OK;
}
