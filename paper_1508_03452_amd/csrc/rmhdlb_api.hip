// rmhdlb_api.hip -- implementation of the C ABI declared in include/rmhdlb.h.
//
// Owns parameter validation, the layout of the device memory of a context
// (two state buffers, scratch, partial sums: one block, the caller's
// workspace or one allocation), the per-run constants and the launch
// sequence.  No host synchronisation except in rmhdlb_moments and the state
// copies.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "rmhdlb.h"
#include "rmhdlb_internal.h"
#include "rmhdlb_mlp.h"

using rmhd::Consts;

// Reduced diagnostics: NPART sums, max |div B|, R, null cell, B0.
constexpr int RESULT_LEN = rmhd::NPART + 4;

struct rmhdlb_ctx {
    rmhdlb_params P;
    hipStream_t stream;
    Consts K;
    int storage;       // RMHDLB_STORE_*
    int device;        // the HIP device current at rmhdlb_create
    void* mem;         // the block every buffer below (to result) is carved from
    bool own_mem;      // mem was allocated by rmhdlb_create (else the caller's workspace)
    bool has_state;    // rmhdlb_init_fields or rmhdlb_set_state has run
    void* buf[2];      // state buffers (distributions, then E_prev and, with the previous-B reading, B_prev)
    rmhd::StateBuf sb[2];
    int cur;
    double* scratch;   // 6 N doubles: initial J0 and E'0, then B and E^z of the moments pass
    double* part;      // per-tile partial diagnostics
    double* part2;     // per-tile max |div B|
    double* nullp;     // per-tile null-point candidates (key, cell)
    double* faceB;     // adjusted normal B of the open-face cells
    double* ez0;       // initial E^z (reconnection rate)
    double* aux;       // aux[0] = max |B| of the initial fields
    double* result;    // NPART sums, max |div B|, R, null cell, B0
    rmhd::GuessTables* gt;  // inference tables of the learned guess (device), null until installed
    double* force;     // external force density, 3 N doubles, null until set
    double* vmax;      // vmax[0]: largest |beta| of the last forced step; then the per-wavefront partials
    int guess_mode;    // RMHDLB_GUESS_*
    int64_t* gate;     // the two slots of the learned guess's gate (rmhd::Consts::gflag_rd)
    int64_t step;
    rmhd::StepTuning tune;
};

// Dispatch on the storage type of a context.
#define RMHD_DISPATCH(C, CALL)                                       \
    ((C)->storage == RMHDLB_STORE_F64 ? rmhd::CALL<double>           \
     : (C)->storage == RMHDLB_STORE_F32 ? rmhd::CALL<float>          \
                                         : rmhd::CALL<_Float16>)

namespace {

// Parameters without the workspace fields.
int validate(const rmhdlb_params* P) {
    if (!P) return RMHDLB_EINVAL;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return RMHDLB_EINVAL;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    if (N > 2147483647LL / 2) return RMHDLB_EINVAL;  // cell indices are 32-bit
    for (int a = 0; a < 3; ++a) {
        const bool lo_ok = P->bc_lo[a] == RMHDLB_BC_PERIODIC || P->bc_lo[a] == RMHDLB_BC_OPEN ||
                           (a == 2 && P->bc_lo[a] == RMHDLB_BC_DRIVEN);
        if (!lo_ok || (P->bc_hi[a] != RMHDLB_BC_PERIODIC && P->bc_hi[a] != RMHDLB_BC_OPEN)) return RMHDLB_EINVAL;
        if ((P->bc_lo[a] == RMHDLB_BC_PERIODIC) != (P->bc_hi[a] == RMHDLB_BC_PERIODIC)) return RMHDLB_EINVAL;
    }
    if (P->divb_fix != 0 && P->divb_fix != 1) return RMHDLB_EINVAL;
    if (P->collision != RMHDLB_COLL_EXPLICIT && P->collision != RMHDLB_COLL_PRINTED) return RMHDLB_EINVAL;
    if (P->flux != RMHDLB_FLUX_MUSCL && P->flux != RMHDLB_FLUX_LAX_WENDROFF) return RMHDLB_EINVAL;
    if (P->b_prev != RMHDLB_BPREV_CURRENT && P->b_prev != RMHDLB_BPREV_PREVIOUS) return RMHDLB_EINVAL;
    if (!(P->dx > 0) || !(P->c > 0) || !(P->mu0 > 0) || !(P->tau > 0) || !(P->alpha >= 0) || !(P->Gamma > 1) ||
        !(P->sigma >= 0) || !(P->nu > 0) || !isfinite(P->sigma) || !isfinite(P->alpha))
        return RMHDLB_EINVAL;
    if (P->storage != RMHDLB_STORE_F64 && P->storage != RMHDLB_STORE_F32 && P->storage != RMHDLB_STORE_F16)
        return RMHDLB_EINVAL;
    for (int k = 0; k < 2; ++k)
        if (P->reserved[k] != 0) return RMHDLB_EINVAL;
    if (P->tau_h != 0.5) return RMHDLB_EUNSUPPORTED;  // the force form of Eq. Ex_force needs tau_h = 1/2
    if (P->b_prev == RMHDLB_BPREV_PREVIOUS && (P->collision != RMHDLB_COLL_EXPLICIT || P->flux != RMHDLB_FLUX_MUSCL))
        return RMHDLB_EUNSUPPORTED;  // the previous-B reading is built with the default collision and faces
    return RMHDLB_OK;
}

// Elements in front of cell 0 of every state array: the two ghost planes of
// a driven low-z face, rounded up so that cell 0 stays 64-element aligned.
int64_t ghost_cells(const Consts& K) { return K.drv ? ((int64_t)2 * K.nx * K.ny + 63) / 64 * 64 : 0; }

Consts make_consts(const rmhdlb_params* P) {
    Consts K;
    memset(&K, 0, sizeof(K));
    K.nx = P->nx;
    K.ny = P->ny;
    K.nz = P->nz;
    for (int a = 0; a < 3; ++a) K.per[a] = P->bc_lo[a] == RMHDLB_BC_PERIODIC ? 1 : 0;
    K.drv = P->bc_lo[2] == RMHDLB_BC_DRIVEN;
    const int dims[3] = {P->nx, P->ny, P->nz};
    int any_open = 0;
    for (int a = 0; a < 3; ++a) {
        K.open_lo[a] = P->divb_fix && dims[a] >= 2 && P->bc_lo[a] == RMHDLB_BC_OPEN;
        K.open_hi[a] = P->divb_fix && dims[a] >= 2 && P->bc_hi[a] == RMHDLB_BC_OPEN;
        any_open |= K.open_lo[a] | K.open_hi[a];
    }
    K.divb = any_open;
    K.band = P->null_band >= 1 ? P->null_band : 64;
    K.coll = P->collision;
    K.flux = P->flux;
    K.bprev = P->b_prev;
    const int64_t fsz[3] = {(int64_t)P->ny * P->nz, (int64_t)P->nx * P->nz, (int64_t)P->nx * P->ny};
    K.fo[0] = 0;
    for (int f = 0; f < 6; ++f) K.fo[f + 1] = K.fo[f] + fsz[f >> 1];
    K.N = (int64_t)P->nx * P->ny * P->nz;
    K.g0 = ghost_cells(K);
    K.stride = (K.g0 + K.N + 63) / 64 * 64;
    const double dt = P->dx / (sqrt(2.0) * P->c);  // dx / dt = sqrt(2) c
    K.c = P->c;
    K.dx = P->dx;
    K.eps0 = 1.0 / (P->mu0 * P->c * P->c);
    K.cour = rmhd::KAPPA * P->c * dt / P->dx;
    K.slope = P->flux == RMHDLB_FLUX_LAX_WENDROFF ? 0.5 * (1.0 - K.cour) : 0.5;
    K.kv = P->alpha * P->c * dt / P->dx;
    K.inv_tau = 1.0 / P->tau;
    const double ct_c0 = sqrt(27.0) / P->nu, ca = sqrt(19.0) / P->nu;
    K.wg = (P->nu / ct_c0) / P->tau;
    K.q = 0.5 * dt * P->mu0 * P->c * P->c;
    K.sigma = P->sigma;
    K.gm1 = P->Gamma - 1.0;
    K.wp[0] = 0.1;
    K.wp[1] = 0.3 - 1.0 / (6.0 * ca * ca);
    K.wp[2] = 1.0 / (12.0 * ca * ca) - 3.0 / 40.0;
    K.gc1 = ct_c0 * 3.0 * ca;
    K.gc2 = ct_c0 * 4.5 * ca * ca;
    K.gc3 = ct_c0 * 1.5;
    K.inv_2dx = 0.5 / P->dx;
    return K;
}

size_t dist_elem(int storage) {
    return storage == RMHDLB_STORE_F64 ? 8 : (storage == RMHDLB_STORE_F32 ? 4 : 2);
}
size_t efield_elem(int storage) { return storage == RMHDLB_STORE_F64 ? 8 : 4; }
// The distribution block: 63 arrays of `stride` values in the pair layout (FP64), 65 in the quad and
// double-quad layouts (FP32, FP16: the rest pair takes a quad with two unused values).
size_t efield_offset(int storage, int64_t stride) {
    const int arrays = rmhd::quad_storage(storage) ? rmhd::QUAD_DIST_ARRAYS : rmhd::PAIR_DIST_ARRAYS;
    const size_t b = (size_t)arrays * (size_t)stride * dist_elem(storage);
    return (b + 255) / 256 * 256;
}
// The field block holds E_prev (3 arrays) and, with the previous-B reading, B_prev (3 more).
size_t buffer_bytes(const Consts& K, int storage) {
    return efield_offset(storage, K.stride) + (size_t)(K.bprev ? 6 : 3) * (size_t)K.stride * efield_elem(storage);
}

// The device memory of a context: the buffers below, each at a 256-byte
// aligned offset of one block.
enum { M_BUF0, M_BUF1, M_SCRATCH, M_PART, M_PART2, M_NULLP, M_FACEB, M_EZ0, M_AUX, M_RESULT, M_GATE, M_COUNT };

size_t mem_layout(const Consts& K, int storage, size_t off[M_COUNT]) {
    const size_t nt = (size_t)rmhd::num_tiles(K);
    const size_t nred = (size_t)((K.N + 255) / 256);  // blocks of the init-reference reduction
    size_t sz[M_COUNT];
    sz[M_BUF0] = sz[M_BUF1] = buffer_bytes(K, storage);
    sz[M_SCRATCH] = sizeof(double) * 6 * (size_t)K.N;  // initial J0 and E'0, then B and E^z of the moments pass
    sz[M_PART] = sizeof(double) * std::max(std::max((size_t)rmhd::NPART * nt, 2 * nred), (size_t)K.nx * K.ny);
    sz[M_PART2] = sizeof(double) * std::max(nt, nred);
    sz[M_NULLP] = sizeof(double) * 2 * nt;
    sz[M_FACEB] = sizeof(double) * (size_t)std::max<int64_t>(K.fo[6], 1);
    sz[M_EZ0] = sizeof(double) * (size_t)K.N;
    sz[M_AUX] = sizeof(double) * 4;
    sz[M_RESULT] = sizeof(double) * RESULT_LEN;
    sz[M_GATE] = sizeof(int64_t) * 3;  // two gate slots, steps that ran the network
    size_t total = 0;
    for (int i = 0; i < M_COUNT; ++i) {
        off[i] = total;
        total += (sz[i] + 255) / 256 * 256;
    }
    return total;
}

// Shifts of the stored f and g: w_i E_ref and w'_i N_ref rounded to the
// arithmetic type (FP32 on the mixed paths), and their exact sums.
void set_shifts(Consts& K, int storage, double eref, double nref) {
    for (int c = 0; c < 3; ++c) K.fsh[c] = K.gsh[c] = 0.0;
    K.fs0 = K.fsaa = K.gs0 = 0.0;
    if (storage == RMHDLB_STORE_F64) return;
    const double w[3] = {rmhd::weight(0), rmhd::weight(1), rmhd::weight(7)};
    for (int c = 0; c < 3; ++c) {
        K.fsh[c] = (double)(float)(w[c] * eref);
        K.gsh[c] = (double)(float)(K.wp[c] * nref);
    }
    K.fs0 = K.fsh[0] + 6.0 * K.fsh[1] + 12.0 * K.fsh[2];
    K.fsaa = 2.0 * K.fsh[1] + 8.0 * K.fsh[2];
    K.gs0 = K.gsh[0] + 6.0 * K.gsh[1] + 12.0 * K.gsh[2];
}

// Per-lane operand tables of the MFMA inference from the flat weights (the
// layouts are those of rmhd::mlp_wave).
void pack_tables(const rmhdlb_guess_weights& W, rmhd::GuessTables& T) {
    using namespace rmhd;
    const float* w = W.w;
    for (int l = 0; l < 64; ++l) {
        const int row = l & 31, h = l >> 5;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * h + j;
            T.a1[l][j] = (_Float16)(k < MLP_IN ? w[OW1 + row * MLP_IN + k] : 0.0f);
        }
        for (int s = 0; s < 2; ++s)
            for (int j = 0; j < 8; ++j) {
                const int k = guess_k(s, j, l);
                T.a2[l][s][j] = (_Float16)w[OW2 + row * 32 + k];
                T.a3[l][s][j] = (_Float16)(row < MLP_OUT ? w[OW3 + row * 32 + k] : 0.0f);
            }
        for (int r = 0; r < 16; ++r) {
            T.b1[l][r] = w[OB1 + mfma_row(r, l)];
            T.b2[l][r] = w[OB2 + mfma_row(r, l)];
        }
    }
    for (int k = 0; k < MLP_OUT; ++k) {
        T.b3[k] = w[OB3 + k];
        T.mu_t[k] = W.mu_t[k];
        T.sd_t[k] = W.sd_t[k];
    }
    for (int j = 0; j < MLP_IN; ++j) {
        T.mu_x[j] = W.mu_x[j];
        T.inv_sd_x[j] = 1.0f / W.sd_x[j];
    }
}

// The step's constants with this step's gate slots: read slot cur (written by
// the previous step), record into the other (record = false: into none).
rmhd::Consts step_consts(const rmhdlb_ctx* C, bool record) {
    rmhd::Consts K = C->K;
    K.gflag_rd = C->gate + C->cur;
    K.gflag_wr = record ? C->gate + (1 - C->cur) : nullptr;
    K.gstep = C->step;
    K.gcount = record ? C->gate + 2 : nullptr;
    return K;
}

// Open the gate of the learned guess for the next step (the network runs until
// a step meets no cell above the flow-ratio gate); with reset, also zero the
// count of steps that ran it.
int arm_gate(rmhdlb_ctx* C, bool reset) {
    int64_t v[3];
    v[C->cur] = C->step - 1;
    v[1 - C->cur] = INT64_MIN;
    v[2] = 0;
    if (hipMemcpyAsync(C->gate, v, (reset ? 3 : 2) * sizeof(int64_t), hipMemcpyHostToDevice, C->stream) !=
            hipSuccess ||
        hipStreamSynchronize(C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    return RMHDLB_OK;
}

int install_guess(rmhdlb_ctx* C, const rmhdlb_guess_weights& W) {
    rmhd::GuessTables* T = new (std::nothrow) rmhd::GuessTables();
    if (!T) return RMHDLB_ENOMEM;
    pack_tables(W, *T);
    int rc = RMHDLB_OK;
    if (!C->gt && hipMalloc((void**)&C->gt, sizeof(rmhd::GuessTables)) != hipSuccess) {
        C->gt = nullptr;
        rc = RMHDLB_ENOMEM;
    } else if (hipMemcpyAsync(C->gt, T, sizeof(rmhd::GuessTables), hipMemcpyHostToDevice, C->stream) != hipSuccess ||
               hipStreamSynchronize(C->stream) != hipSuccess) {
        rc = RMHDLB_EDEVICE;
    }
    delete T;
    return rc;
}

// Device buffers of one training run, freed together.
struct TrainBufs {
    double *F = nullptr, *T = nullptr, *part = nullptr;
    float *X = nullptr, *Y = nullptr, *w = nullptr, *m = nullptr, *v = nullptr, *losses = nullptr;
    ~TrainBufs() {
        for (void* p : {(void*)F, (void*)T, (void*)part, (void*)X, (void*)Y, (void*)w, (void*)m, (void*)v,
                        (void*)losses})
            if (p) (void)hipFree(p);
    }
};

template <typename Tp>
bool dalloc(Tp** p, size_t n) {
    if (hipMalloc((void**)p, sizeof(Tp) * (n > 0 ? n : 1)) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    return true;
}

void release(rmhdlb_ctx* C) {
    if (!C) return;
    if (C->own_mem && C->mem) (void)hipFree(C->mem);
    if (C->gt) (void)hipFree(C->gt);
    if (C->force) (void)hipFree(C->force);
    if (C->vmax) (void)hipFree(C->vmax);
    delete C;
}

}  // namespace

extern "C" {

const char* rmhdlb_strerror(int code) {
    switch (code) {
        case RMHDLB_OK: return "ok";
        case RMHDLB_EINVAL: return "invalid argument";
        case RMHDLB_ENOMEM: return "device allocation failed";
        case RMHDLB_EDEVICE: return "HIP runtime or launch error";
        case RMHDLB_ERECOVERY: return "primitive recovery failed in some cells";
        case RMHDLB_EUNSUPPORTED: return "unsupported parameter value";
        case RMHDLB_ESTATE: return "call out of order (no state yet, or batch instances at different time levels)";
        case RMHDLB_ELIMIT: return "size beyond the fixed device memory of a no-allocation entry point";
        default: return "unknown error";
    }
}

size_t rmhdlb_workspace_bytes(const rmhdlb_params* params) {
    if (validate(params) != RMHDLB_OK) return 0;
    size_t off[M_COUNT];
    return mem_layout(make_consts(params), params->storage, off);
}

int rmhdlb_create(const rmhdlb_params* params, void* hip_stream, rmhdlb_ctx** out) {
    if (!out) return RMHDLB_EINVAL;
    *out = nullptr;
    const int v = validate(params);
    if (v != RMHDLB_OK) return v;
    const Consts K = make_consts(params);
    size_t off[M_COUNT];
    const size_t total = mem_layout(K, params->storage, off);
    if (params->workspace && (params->workspace_bytes < total || ((uintptr_t)params->workspace & 255) != 0))
        return RMHDLB_EINVAL;
    rmhdlb_ctx* C = new (std::nothrow) rmhdlb_ctx();
    if (!C) return RMHDLB_ENOMEM;
    C->P = *params;
    C->stream = (hipStream_t)hip_stream;
    C->K = K;
    if (hipGetDevice(&C->device) != hipSuccess) {
        release(C);
        return RMHDLB_EDEVICE;
    }
    C->storage = params->storage;
    if (params->workspace) {
        C->mem = params->workspace;
        C->own_mem = false;
    } else if (hipMalloc(&C->mem, total) != hipSuccess) {
        (void)hipGetLastError();
        C->mem = nullptr;
        release(C);
        return RMHDLB_ENOMEM;
    } else {
        C->own_mem = true;
    }
    // cleared once so that ghost planes and padding hold defined values
    if (hipMemsetAsync(C->mem, 0, total, C->stream) != hipSuccess) {
        release(C);
        return RMHDLB_EDEVICE;
    }
    char* base = (char*)C->mem;
    const int64_t g0 = ghost_cells(C->K);
    for (int b = 0; b < 2; ++b) {
        C->buf[b] = base + off[M_BUF0 + b];
        C->sb[b].dist = (char*)C->buf[b] + g0 * dist_elem(C->storage);
        C->sb[b].efield = (char*)C->buf[b] + efield_offset(C->storage, C->K.stride) + g0 * efield_elem(C->storage);
    }
    C->scratch = (double*)(base + off[M_SCRATCH]);
    C->part = (double*)(base + off[M_PART]);
    C->part2 = (double*)(base + off[M_PART2]);
    C->nullp = (double*)(base + off[M_NULLP]);
    C->faceB = (double*)(base + off[M_FACEB]);
    C->ez0 = (double*)(base + off[M_EZ0]);
    C->aux = (double*)(base + off[M_AUX]);
    C->result = (double*)(base + off[M_RESULT]);
    C->gate = (int64_t*)(base + off[M_GATE]);
    C->K.gflag_rd = nullptr;
    C->K.gflag_wr = nullptr;
    C->K.gstep = 0;
    C->K.gcount = nullptr;
    C->has_state = false;
    C->cur = 0;
    C->step = 0;
    // Launch shape until rmhdlb_autotune or rmhdlb_set_tuning picks another.
    C->tune.zb = 4;
    C->tune.px = 64;
    C->tune.zg = 1;
    *out = C;
    return RMHDLB_OK;
}

int rmhdlb_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return RMHDLB_EINVAL;
    const uintptr_t d = (uintptr_t)dst, s0 = (uintptr_t)src;
    if (d < s0 + bytes && s0 < d + bytes) return RMHDLB_EINVAL;  // overlapping
    return rmhd::launch_copy16(src, dst, (int64_t)(bytes / 16), (hipStream_t)hip_stream) == hipSuccess
               ? RMHDLB_OK
               : RMHDLB_EDEVICE;
}

int rmhdlb_destroy(rmhdlb_ctx* ctx) {
    if (!ctx) return RMHDLB_OK;
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    return RMHDLB_OK;
}

int rmhdlb_init_fields(rmhdlb_ctx* C, const rmhdlb_fields_in* in) {
    if (!C || !in || !in->n || !in->p) return RMHDLB_EINVAL;
    rmhd::InPtrs ip;
    ip.n = in->n;
    ip.p = in->p;
    for (int a = 0; a < 3; ++a) {
        if (!in->u[a] || !in->E[a] || !in->B[a]) return RMHDLB_EINVAL;
        ip.u[a] = in->u[a];
        ip.E[a] = in->E[a];
        ip.B[a] = in->B[a];
    }
    ip.rho_c = in->rho_c;
    C->cur = 0;
    if (C->storage != RMHDLB_STORE_F64) {
        // references of the stored deviations: means of eps and n over the initial fields
        if (rmhd::launch_init_ref(ip, C->K, C->part, C->result, C->stream) != hipSuccess) return RMHDLB_EDEVICE;
        double r[2];
        if (hipMemcpyAsync(r, C->result, sizeof(r), hipMemcpyDeviceToHost, C->stream) != hipSuccess ||
            hipStreamSynchronize(C->stream) != hipSuccess)
            return RMHDLB_EDEVICE;
        set_shifts(C->K, C->storage, r[0] / (double)C->K.N, r[1] / (double)C->K.N);
    } else {
        set_shifts(C->K, C->storage, 0.0, 0.0);
    }
    hipError_t e = RMHD_DISPATCH(C, launch_init)(ip, C->K, C->scratch, C->sb[0], C->stream);
    if (e != hipSuccess) return RMHDLB_EDEVICE;
    // references of the reconnection rate: E^z_0 and B0 = max |B|
    if (hipMemcpyAsync(C->ez0, in->E[2], sizeof(double) * (size_t)C->K.N, hipMemcpyDeviceToDevice, C->stream) !=
            hipSuccess ||
        rmhd::launch_init_bmax(ip, C->K, C->part2, C->aux, C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    // a driven face starts from the fields of the first interior plane
    if (C->K.drv) {
        rmhd::FacePtrs fp;
        fp.n = in->n;
        fp.p = in->p;
        for (int a = 0; a < 3; ++a) {
            fp.u[a] = in->u[a];
            fp.B[a] = in->B[a];
        }
        for (int b = 0; b < 2; ++b)
            if (RMHD_DISPATCH(C, launch_ghost)(fp, C->K, C->sb[b], C->stream) != hipSuccess) return RMHDLB_EDEVICE;
    }
    if (C->K.forced && hipMemsetAsync(C->vmax, 0, sizeof(double), C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;  // the force gate starts open
    C->step = 0;
    C->has_state = true;
    return arm_gate(C, true);
}

int rmhdlb_set_force(rmhdlb_ctx* C, const double* const F[3], double gate) {
    if (!C || !isfinite(gate)) return RMHDLB_EINVAL;
    if (!F) {
        C->K.forced = 0;
        return RMHDLB_OK;
    }
    for (int a = 0; a < 3; ++a)
        if (!F[a]) return RMHDLB_EINVAL;
    if (C->K.flux || C->guess_mode || C->K.bprev) return RMHDLB_EUNSUPPORTED;
    const int64_t N = C->K.N;
    // one partial per wavefront of the widest launch (64-wide tiles, one plane per block)
    const int64_t nparts = 4 * (int64_t)((C->K.nx + 63) / 64) * ((C->K.ny + 1) / 2) * C->K.nz;
    if (!C->force && hipMalloc((void**)&C->force, sizeof(double) * 3 * (size_t)N) != hipSuccess) {
        C->force = nullptr;
        return RMHDLB_ENOMEM;
    }
    if (!C->vmax && hipMalloc((void**)&C->vmax, sizeof(double) * (size_t)(1 + nparts)) != hipSuccess) {
        C->vmax = nullptr;
        return RMHDLB_ENOMEM;
    }
    for (int a = 0; a < 3; ++a)
        if (hipMemcpyAsync(C->force + a * N, F[a], sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, C->stream) !=
            hipSuccess)
            return RMHDLB_EDEVICE;
    if (hipMemsetAsync(C->vmax, 0, sizeof(double) * (size_t)(1 + nparts), C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    C->K.force = C->force;
    C->K.vmax_prev = C->vmax;
    C->K.vmax_part = C->vmax + 1;
    C->K.fgate = gate;
    C->K.forced = 1;
    return RMHDLB_OK;
}

int rmhdlb_set_driven_face(rmhdlb_ctx* C, const rmhdlb_face_in* face) {
    if (!C || !face || !face->n || !face->p || !C->K.drv) return RMHDLB_EINVAL;
    rmhd::FacePtrs fp;
    fp.n = face->n;
    fp.p = face->p;
    for (int a = 0; a < 3; ++a) {
        if (!face->u[a] || !face->B[a]) return RMHDLB_EINVAL;
        fp.u[a] = face->u[a];
        fp.B[a] = face->B[a];
    }
    double bad = 0.0;
    if (rmhd::launch_face_check(fp, C->K, C->part, C->result, C->stream) != hipSuccess ||
        hipMemcpyAsync(&bad, C->result, sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess ||
        hipStreamSynchronize(C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    if (bad != 0.0) return RMHDLB_EINVAL;
    for (int b = 0; b < 2; ++b)
        if (RMHD_DISPATCH(C, launch_ghost)(fp, C->K, C->sb[b], C->stream) != hipSuccess) return RMHDLB_EDEVICE;
    return RMHDLB_OK;
}

int rmhdlb_step(rmhdlb_ctx* C, int64_t nsteps) {
    if (!C || nsteps < 0) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    for (int64_t s = 0; s < nsteps; ++s) {
        hipError_t e = RMHD_DISPATCH(C, launch_step)(C->sb[C->cur], C->sb[1 - C->cur], step_consts(C, true), C->tune,
                                                     C->faceB, C->guess_mode ? C->gt : nullptr, C->stream);
        if (e != hipSuccess) return RMHDLB_EDEVICE;
        C->cur = 1 - C->cur;
        C->step++;
    }
    return RMHDLB_OK;
}

int rmhdlb_moments(rmhdlb_ctx* C, rmhdlb_fields_out* out, rmhdlb_diag* diag) {
    if (!C) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    rmhd::OutPtrs op;
    memset(&op, 0, sizeof(op));
    if (out) {
        op.n = out->n;
        op.p = out->p;
        op.eps = out->eps;
        for (int a = 0; a < 3; ++a) {
            op.u[a] = out->u[a];
            op.E[a] = out->E[a];
            op.B[a] = out->B[a];
            op.J[a] = out->J[a];
        }
        op.rho_c = out->rho_c;
    }
    rmhd::DiagBufs D;
    D.faceB = C->faceB;
    D.scratch = C->scratch;
    D.part = C->part;
    D.part2 = C->part2;
    D.nullp = C->nullp;
    D.ez0 = C->ez0;
    D.b0 = C->aux;
    D.result = C->result;
    hipError_t e = RMHD_DISPATCH(C, launch_moments)(C->sb[C->cur], step_consts(C, false), op, D,
                                                    C->guess_mode ? C->gt : nullptr, C->stream);
    if (e != hipSuccess) return RMHDLB_EDEVICE;
    double r[RESULT_LEN];
    int64_t guess_steps = 0;
    if (hipMemcpyAsync(r, C->result, sizeof(r), hipMemcpyDeviceToHost, C->stream) != hipSuccess ||
        hipMemcpyAsync(&guess_steps, C->gate + 2, sizeof(int64_t), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    if (hipStreamSynchronize(C->stream) != hipSuccess) return RMHDLB_EDEVICE;
    const int64_t failed = (int64_t)llround(r[8]);
    if (diag) {
        diag->energy = r[0];
        diag->mass = r[1];
        diag->momentum[0] = r[2];
        diag->momentum[1] = r[3];
        diag->momentum[2] = r[4];
        diag->em_energy = r[5];
        diag->charge = r[6];
        diag->mean_iters = r[7] / (double)C->K.N;
        for (int k = 0; k < 16; ++k) diag->newton_hist[k] = (int64_t)llround(r[9 + k]);
        diag->n_failed = failed;
        diag->n_fallback = (int64_t)llround(r[25]);
        diag->max_divB = r[rmhd::NPART];
        diag->recon_rate = r[rmhd::NPART + 1];
        diag->null_index = (int64_t)llround(r[rmhd::NPART + 2]);
        diag->B0 = r[rmhd::NPART + 3];
        diag->step = C->step;
        diag->guess_steps = guess_steps;
    }
    return failed ? RMHDLB_ERECOVERY : RMHDLB_OK;
}

int rmhdlb_set_guess_weights(rmhdlb_ctx* C, const rmhdlb_guess_weights* w) {
    if (!C || !w) return RMHDLB_EINVAL;
    for (int j = 0; j < 6; ++j)
        if (!(w->sd_x[j] > 0.0f)) return RMHDLB_EINVAL;
    return install_guess(C, *w);
}

int rmhdlb_set_guess(rmhdlb_ctx* C, int32_t mode) {
    if (!C || (mode != RMHDLB_GUESS_PLAIN && mode != RMHDLB_GUESS_MLP)) return RMHDLB_EINVAL;
    if (mode == RMHDLB_GUESS_MLP && !C->gt) return RMHDLB_EINVAL;
    if (mode == RMHDLB_GUESS_MLP && (C->K.coll || C->K.flux || C->K.forced || C->K.bprev))
        return RMHDLB_EUNSUPPORTED;  // default readings, no force
    C->guess_mode = mode;
    return mode == RMHDLB_GUESS_MLP && C->has_state ? arm_gate(C, false) : RMHDLB_OK;
}

static int sample_cells(rmhdlb_ctx* C, int ns, double* F, double* T, double* part, double sums[rmhd::SAMPLE_SUMS]) {
    hipError_t e = RMHD_DISPATCH(C, launch_guess_samples)(C->sb[C->cur], C->K, C->faceB, ns, F, T, part, C->result,
                                                          C->stream);
    if (e != hipSuccess ||
        hipMemcpyAsync(sums, C->result, sizeof(double) * rmhd::SAMPLE_SUMS, hipMemcpyDeviceToHost, C->stream) !=
            hipSuccess ||
        hipStreamSynchronize(C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    return sums[16] != 0.0 ? RMHDLB_ERECOVERY : RMHDLB_OK;
}

int rmhdlb_guess_samples(rmhdlb_ctx* C, int32_t ns, double* F, double* T) {
    if (!C || !F || !T || ns < 1 || ns > C->K.N) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    if (C->K.bprev) return RMHDLB_EUNSUPPORTED;
    double* part = nullptr;
    if (!dalloc(&part, (size_t)rmhd::SAMPLE_SUMS * ((ns + 255) / 256))) return RMHDLB_ENOMEM;
    double sums[rmhd::SAMPLE_SUMS];
    const int rc = sample_cells(C, ns, F, T, part, sums);
    (void)hipFree(part);
    return rc;
}

}  // extern "C"

// ------------------------------------------------ the no-allocation entry point

// Per-block partial sums of the sampling pass of rmhdlb_guess_samples_noalloc:
// one fixed array per device, which the host reaches only through the address
// hipGetSymbolAddress returns for that device (kept in g_scratch_ptr); the
// array's own name is no device address in host code.
constexpr size_t NOALLOC_SCRATCH_LEN = (size_t)rmhd::SAMPLE_SUMS * ((RMHDLB_NOALLOC_MAX_SAMPLES + 255) / 256);
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_LEN];

namespace {

std::mutex g_scratch_mutex;
std::map<int, double*> g_scratch_ptr;  // device -> address of its copy of `scratch`

// The address of device dev's copy of `scratch`, resolved once per device
// with that device current (the caller's current device is restored).
int scratch_on_device(int dev, double** out) {
    std::lock_guard<std::mutex> g(g_scratch_mutex);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return RMHDLB_OK;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return RMHDLB_EDEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return RMHDLB_EDEVICE;
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return RMHDLB_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
    *out = p;
    return RMHDLB_OK;
}

}  // namespace

extern "C" {

int rmhdlb_guess_samples_noalloc(rmhdlb_ctx* C, int32_t ns, double* F, double* T) {
    if (!C || !F || !T || ns < 1) return RMHDLB_EINVAL;
    if (ns > RMHDLB_NOALLOC_MAX_SAMPLES) return RMHDLB_ELIMIT;
    if (ns > C->K.N) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    if (C->K.bprev) return RMHDLB_EUNSUPPORTED;
    double* part = nullptr;
    const int rc = scratch_on_device(C->device, &part);
    if (rc != RMHDLB_OK) return rc;
    double sums[rmhd::SAMPLE_SUMS];
    return sample_cells(C, ns, F, T, part, sums);
}

int rmhdlb_train_guess(rmhdlb_ctx* C, const rmhdlb_train_opts* o, const float* init_w, rmhdlb_guess_weights* out,
                       float* losses) {
    if (!C || !o || !init_w) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    if (C->K.bprev) return RMHDLB_EUNSUPPORTED;
    const int ns = o->n_samples;
    if (ns < 128 || ns > C->K.N || o->batch < 128 || o->batch % 128 != 0 || o->batch > ns || o->iters < 0 ||
        o->stride < 1 || !(o->lr > 0.0f) || !isfinite(o->lr) || o->reserved[0] || o->reserved[1] || o->reserved[2])
        return RMHDLB_EINVAL;
    TrainBufs B;
    const int np = rmhd::MLP_NP;
    if (!dalloc(&B.F, (size_t)ns * 6) || !dalloc(&B.T, (size_t)ns * 2) ||
        !dalloc(&B.part, (size_t)rmhd::SAMPLE_SUMS * ((ns + 255) / 256)) || !dalloc(&B.X, (size_t)ns * 6) ||
        !dalloc(&B.Y, (size_t)ns * 2) || !dalloc(&B.w, np) || !dalloc(&B.m, np) || !dalloc(&B.v, np) ||
        !dalloc(&B.losses, (size_t)o->iters))
        return RMHDLB_ENOMEM;
    double sums[rmhd::SAMPLE_SUMS];
    int rc = sample_cells(C, ns, B.F, B.T, B.part, sums);
    if (rc != RMHDLB_OK) return rc;
    // normalisation: sample mean and (population) standard deviation, floor 1e-6
    rmhd::Norm4 nm;
    rmhdlb_guess_weights W;
    for (int j = 0; j < 8; ++j) {
        const double mu = (j < 6 ? sums[j] : sums[12 + (j - 6)]) / ns;
        const double sq = (j < 6 ? sums[6 + j] : sums[14 + (j - 6)]) / ns;
        const double sd = fmax(sqrt(fmax(sq - mu * mu, 0.0)), 1e-6);
        if (j < 6) {
            nm.mu_x[j] = mu;
            nm.sd_x[j] = sd;
            W.mu_x[j] = (float)mu;
            W.sd_x[j] = (float)sd;
        } else {
            nm.mu_t[j - 6] = mu;
            nm.sd_t[j - 6] = sd;
            W.mu_t[j - 6] = (float)mu;
            W.sd_t[j - 6] = (float)sd;
        }
    }
    if (rmhd::launch_guess_normalise(B.F, B.T, ns, nm, B.X, B.Y, C->stream) != hipSuccess ||
        hipMemcpyAsync(B.w, init_w, sizeof(float) * np, hipMemcpyHostToDevice, C->stream) != hipSuccess ||
        hipMemsetAsync(B.m, 0, sizeof(float) * np, C->stream) != hipSuccess ||
        hipMemsetAsync(B.v, 0, sizeof(float) * np, C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    rmhd::TrainArgs A;
    memset(&A, 0, sizeof(A));
    A.X = B.X;
    A.Yt = B.Y;
    A.n = ns;
    A.batch = o->batch;
    A.iters = o->iters;
    A.stride = o->stride;
    A.lr = o->lr;
    A.w = B.w;
    A.m = B.m;
    A.v = B.v;
    A.losses = B.losses;
    if (rmhd::launch_train(A, C->stream) != hipSuccess ||
        hipMemcpyAsync(W.w, B.w, sizeof(float) * np, hipMemcpyDeviceToHost, C->stream) != hipSuccess ||
        (losses && o->iters > 0 &&
         hipMemcpyAsync(losses, B.losses, sizeof(float) * o->iters, hipMemcpyDeviceToHost, C->stream) != hipSuccess) ||
        hipStreamSynchronize(C->stream) != hipSuccess)
        return RMHDLB_EDEVICE;
    rc = install_guess(C, W);
    if (rc == RMHDLB_OK && out) *out = W;
    return rc;
}

int rmhdlb_mlp_eval(const float* w, const float* X, const float* Yt, int32_t n, float* Y, float* grad, float* loss,
                    void* hip_stream) {
    if (!w || !X || !Yt || !grad || !loss || n < 128 || n % 128 != 0 || n > 65536) return RMHDLB_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    float* wd = nullptr;
    if (!dalloc(&wd, rmhd::MLP_NP)) return RMHDLB_ENOMEM;
    rmhd::TrainArgs A;
    memset(&A, 0, sizeof(A));
    A.X = X;
    A.Yt = Yt;
    A.n = n;
    A.batch = n;
    A.iters = 1;
    A.stride = 1;
    A.lr = 0.0f;
    A.w = wd;
    A.losses = loss;
    A.grad = grad;
    A.y = Y;
    A.grad_only = 1;
    int rc = RMHDLB_OK;
    if (hipMemcpyAsync(wd, w, sizeof(float) * rmhd::MLP_NP, hipMemcpyHostToDevice, st) != hipSuccess ||
        rmhd::launch_train(A, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        rc = RMHDLB_EDEVICE;
    (void)hipFree(wd);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------- tuning

namespace {

// nx, ny, nz, storage, divb, driven, guess, collision, flux, force, previous B
typedef std::tuple<int, int, int, int, int, int, int, int, int, int, int> TuneKey;
std::map<TuneKey, rmhd::StepTuning> g_tune_cache;
std::mutex g_tune_mutex;

// Average duration (ms) of `reps` calls of fn on the stream after one warm-up.
template <typename Fn>
int time_ms(hipStream_t st, int reps, Fn fn, float* ms) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return RMHDLB_EDEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return RMHDLB_EDEVICE;
    }
    int rc = fn() == hipSuccess ? RMHDLB_OK : RMHDLB_EDEVICE;
    if (rc == RMHDLB_OK && hipEventRecord(a, st) != hipSuccess) rc = RMHDLB_EDEVICE;
    for (int r = 0; r < reps && rc == RMHDLB_OK; ++r)
        if (fn() != hipSuccess) rc = RMHDLB_EDEVICE;
    if (rc == RMHDLB_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                            hipEventElapsedTime(ms, a, b) != hipSuccess))
        rc = RMHDLB_EDEVICE;
    *ms /= reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

}  // namespace

extern "C" {

int rmhdlb_autotune(rmhdlb_ctx* C, int32_t* px_out, int32_t* zb_out, int32_t* zg_out, int32_t* yw_out) {
    if (!C) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    const TuneKey key(C->K.nx, C->K.ny, C->K.nz, C->storage, C->K.divb, C->K.drv, C->guess_mode, C->K.coll,
                      C->K.flux, C->K.forced, C->K.bprev);
    rmhd::StepTuning best;
    best.px = 64;
    best.zb = 4;
    best.zg = 1;
    best.yw = 1;
    bool cached = false;
    {
        std::lock_guard<std::mutex> g(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best = it->second;
            cached = true;
        }
    }
    if (!cached) {
        // Candidates: every tile width with zb in {1, 2, 4, 8, 16} walked by
        // one block, and 64-wide tiles with long walks shared by 2 or 4
        // interleaved blocks per column (chunks of up to 256 planes).  On a
        // slab (nz = 1) the blocks instead take 1, 2 or 4 row groups.
        std::vector<rmhd::StepTuning> cand;
        const bool only64 = C->guess_mode || C->K.coll || C->K.flux || C->K.forced || C->K.bprev;
        for (int px : {64, 32, 16})
            for (int zb : {1, 2, 4, 8, 16})
                for (int yw : {1, 2, 4}) {
                    if ((zb > C->K.nz && zb != 1) || (only64 && px != 64)) continue;
                    if (yw > 1 && (C->K.nz > 1 || C->K.forced)) continue;
                    rmhd::StepTuning t;
                    t.px = px;
                    t.zb = zb;
                    t.zg = 1;
                    t.yw = yw;
                    cand.push_back(t);
                }
        if (!C->K.forced)
            for (int zg : {2, 4})
                for (int zb : {16, 32, 64}) {
                    if (zg * zb > C->K.nz) continue;
                    rmhd::StepTuning t;
                    t.px = 64;
                    t.zb = zb;
                    t.zg = zg;
                    cand.push_back(t);
                }
        // A forced step also reduces its largest |beta| into the gate's
        // lagged value: keep the value of the last real step across the timing.
        double gate_prev = 0.0;
        if (C->K.forced && (hipMemcpyAsync(&gate_prev, C->K.vmax_prev, sizeof(double), hipMemcpyDeviceToHost,
                                           C->stream) != hipSuccess ||
                            hipStreamSynchronize(C->stream) != hipSuccess))
            return RMHDLB_EDEVICE;
        float best_ms = 1e30f;
        for (const rmhd::StepTuning& t : cand) {
            float ms = 0.0f;
            const int rc = time_ms(C->stream, 3, [&]() {
                // the trials read the gate slot of this step and record into the slot this step will record
                // into, with this step's number and from this step's state: what the real step records
                rmhd::Consts Kt = step_consts(C, true);
                Kt.gcount = nullptr;  // trials are not steps
                return RMHD_DISPATCH(C, launch_step)(C->sb[C->cur], C->sb[1 - C->cur], Kt, t, C->faceB,
                                                     C->guess_mode ? C->gt : nullptr, C->stream);
            }, &ms);
            if (rc != RMHDLB_OK) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        if (C->K.forced && (hipMemcpyAsync(const_cast<double*>(C->K.vmax_prev), &gate_prev, sizeof(double),
                                           hipMemcpyHostToDevice, C->stream) != hipSuccess ||
                            hipStreamSynchronize(C->stream) != hipSuccess))
            return RMHDLB_EDEVICE;
        std::lock_guard<std::mutex> g(g_tune_mutex);
        g_tune_cache[key] = best;
    }
    C->tune = best;
    if (px_out) *px_out = best.px;
    if (zb_out) *zb_out = best.zb;
    if (zg_out) *zg_out = best.zg;
    if (yw_out) *yw_out = best.yw;
    return RMHDLB_OK;
}

int rmhdlb_set_tuning(rmhdlb_ctx* C, int32_t px, int32_t zb, int32_t zg, int32_t yw) {
    if (!C || (px != 64 && px != 32 && px != 16) || zb < 1 || zg < 1 || zg > 64 || yw < 1 || yw > 8)
        return RMHDLB_EINVAL;
    if ((C->guess_mode || C->K.coll || C->K.flux || C->K.forced || C->K.bprev) && px != 64) return RMHDLB_EINVAL;
    if (C->K.forced && (zg != 1 || yw != 1)) return RMHDLB_EINVAL;
    // More blocks per column than the chunk has planes would only walk
    // nothing: cap zg at ceil(nz / zb) (zb as the step clamps it to nz),
    // which also keeps zg * zb within int range.
    const int zbe = zb < C->K.nz ? zb : C->K.nz;
    const int zg_max = (C->K.nz + zbe - 1) / zbe;
    C->tune.px = px;
    C->tune.zb = zb;
    C->tune.zg = zg < zg_max ? zg : zg_max;
    C->tune.yw = yw;
    return RMHDLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches

// Steps per captured graph of a batch: long replays for long sweeps, a
// two-step graph for the rest (each starts and ends at buffer parity 0).
constexpr int GRAPH_LONG = 64;

// Launch dimensions baked into a captured graph: the graph must be captured
// again when any of them changes.
struct BatchGeom {
    int px = 0, yw = 0, waves = 0, total_blocks = -1;
    int64_t total_face = -1;
    bool operator==(const BatchGeom& o) const {
        return px == o.px && yw == o.yw && waves == o.waves && total_blocks == o.total_blocks &&
               total_face == o.total_face;
    }
};

struct rmhdlb_batch {
    int n;
    std::vector<rmhdlb_ctx*> ctx;
    hipStream_t stream;
    int storage;
    int px;     // tile width (128, 64, 32, 16)
    int yw;     // row groups per block (the tile is px x (128 / px) yw cells on a slab)
    int waves;  // occupancy variant of the FP32 kernel (2 or 3 waves per SIMD)
    std::vector<rmhd::BatchInst> host;
    rmhd::BatchInst* dev;
    int total_blocks;
    int64_t total_face;
    int persistent;            // rmhdlb_batch_step: 1 = one cooperative launch per call
    int* next;                 // the persistent kernel's tile counters (after the instance table)
    hipGraphExec_t exec_long;  // GRAPH_LONG steps from parity 0, or null
    hipGraphExec_t exec_pair;  // two steps from parity 0, or null
    BatchGeom graph_geom;      // the geometry both graphs were captured with
};

namespace {

BatchGeom batch_geom(const rmhdlb_batch* B) {
    BatchGeom g;
    g.px = B->px;
    g.yw = B->yw;
    g.waves = B->waves;
    g.total_blocks = B->total_blocks;
    g.total_face = B->total_face;
    return g;
}

// Per-instance table of the batched launches from the instances' current
// constants and buffers.
int batch_table(rmhdlb_batch* B) {
    int64_t blk = 0, face = 0;
    for (int i = 0; i < B->n; ++i) {
        rmhdlb_ctx* C = B->ctx[i];
        rmhd::BatchInst& I = B->host[i];
        I.K = C->K;
        for (int b = 0; b < 2; ++b) {
            I.dist[b] = C->sb[b].dist;
            I.efield[b] = C->sb[b].efield;
        }
        I.faceB = C->faceB;
        I.zb = std::max(1, std::min(C->tune.zb, C->K.nz));
        I.yw = B->yw;
        rmhd::step_geometry(C->K, B->px, I.zb, 1, I.yw, rmhd::cells_per_block(rmhd::quad_storage(B->storage)),
                            I.tiles_x, I.ncol, I.nblk);
        I.blk0 = blk;
        I.face0 = face;
        blk += I.nblk;
        face += C->K.divb ? C->K.fo[6] : 0;
    }
    if (blk > 2147483647LL - 8) return RMHDLB_EINVAL;
    B->total_blocks = (int)blk;
    B->total_face = face;
    return hipMemcpyAsync(B->dev, B->host.data(), sizeof(rmhd::BatchInst) * B->n, hipMemcpyHostToDevice, B->stream) ==
                   hipSuccess
               ? RMHDLB_OK
               : RMHDLB_EDEVICE;
}

hipError_t batch_launch(rmhdlb_batch* B, int parity) {
    switch (B->storage) {
        case RMHDLB_STORE_F64:
            return rmhd::launch_batch<double>(B->dev, B->n, B->total_blocks, B->total_face, B->px, B->waves, parity,
                                              B->stream);
        case RMHDLB_STORE_F32:
            return rmhd::launch_batch<float>(B->dev, B->n, B->total_blocks, B->total_face, B->px, B->waves, parity,
                                             B->stream);
        default:
            return rmhd::launch_batch<_Float16>(B->dev, B->n, B->total_blocks, B->total_face, B->px, B->waves,
                                                parity, B->stream);
    }
}

hipError_t batch_launch_persistent(rmhdlb_batch* B, int parity, int nsteps) {
    switch (B->storage) {
        case RMHDLB_STORE_F64:
            return rmhd::launch_batch_persistent<double>(B->dev, B->n, B->total_blocks, B->px, B->waves,
                                                         parity, nsteps, B->next, B->stream);
        case RMHDLB_STORE_F32:
            return rmhd::launch_batch_persistent<float>(B->dev, B->n, B->total_blocks, B->px, B->waves,
                                                        parity, nsteps, B->next, B->stream);
        default:
            return rmhd::launch_batch_persistent<_Float16>(B->dev, B->n, B->total_blocks, B->px, B->waves,
                                                           parity, nsteps, B->next, B->stream);
    }
}

void drop_graphs(rmhdlb_batch* B) {
    if (B->exec_long) (void)hipGraphExecDestroy(B->exec_long);
    if (B->exec_pair) (void)hipGraphExecDestroy(B->exec_pair);
    B->exec_long = B->exec_pair = nullptr;
}

// Capture nsteps (even) steps from parity 0 into an executable graph; null
// on any failure (the batch then steps eagerly).
hipGraphExec_t capture_steps(rmhdlb_batch* B, int nsteps) {
    if (!B->stream) return nullptr;  // the legacy default stream cannot be captured
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    bool ok = true;
    for (int k = 0; k < nsteps && ok; ++k) ok = batch_launch(B, k & 1) == hipSuccess;
    if (hipStreamEndCapture(B->stream, &g) != hipSuccess || !ok || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return nullptr;
    }
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        e = nullptr;
    }
    (void)hipGraphDestroy(g);
    return e;
}

int check_batch_state(rmhdlb_batch* B) {
    const int parity0 = B->ctx[0]->cur;
    for (rmhdlb_ctx* C : B->ctx) {
        if (!C->has_state || C->cur != parity0) return RMHDLB_ESTATE;
        if (C->guess_mode || C->K.forced) return RMHDLB_EUNSUPPORTED;
    }
    return RMHDLB_OK;
}

// Batch tuning cache: storage and every instance's grid.
typedef std::pair<int, std::vector<std::tuple<int, int, int>>> BatchKey;
struct BatchShape {
    int px, yw, waves;
};
std::map<BatchKey, BatchShape> g_batch_cache;

}  // namespace

extern "C" {

int rmhdlb_batch_create(const rmhdlb_params* params, int32_t n, void* hip_stream, rmhdlb_batch** out) {
    if (!out) return RMHDLB_EINVAL;
    *out = nullptr;
    if (!params || n < 1) return RMHDLB_EINVAL;
    for (int i = 1; i < n; ++i)
        if (params[i].storage != params[0].storage) return RMHDLB_EINVAL;
    for (int i = 0; i < n; ++i)
        if (params[i].collision != RMHDLB_COLL_EXPLICIT || params[i].flux != RMHDLB_FLUX_MUSCL ||
            params[i].b_prev != RMHDLB_BPREV_CURRENT)
            return RMHDLB_EUNSUPPORTED;  // batches: the default readings only
    rmhdlb_batch* B = new (std::nothrow) rmhdlb_batch();
    if (!B) return RMHDLB_ENOMEM;
    B->n = n;
    B->stream = (hipStream_t)hip_stream;
    B->storage = params[0].storage;
    B->px = 64;
    B->yw = 1;
    B->waves = 2;
    B->persistent = 0;
    B->dev = nullptr;
    B->next = nullptr;
    B->exec_long = B->exec_pair = nullptr;
    B->total_blocks = 0;
    B->total_face = 0;
    B->ctx.assign(n, nullptr);
    B->host.resize(n);
    int rc = RMHDLB_OK;
    for (int i = 0; i < n && rc == RMHDLB_OK; ++i) rc = rmhdlb_create(&params[i], hip_stream, &B->ctx[i]);
    // the instance table, then the persistent kernel's 16 tile counters
    const size_t table = (sizeof(rmhd::BatchInst) * n + 255) / 256 * 256;
    if (rc == RMHDLB_OK && hipMalloc((void**)&B->dev, table + 16 * sizeof(int)) != hipSuccess) {
        B->dev = nullptr;
        rc = RMHDLB_ENOMEM;
    }
    if (rc != RMHDLB_OK) {
        rmhdlb_batch_destroy(B);
        return rc;
    }
    B->next = reinterpret_cast<int*>(reinterpret_cast<char*>(B->dev) + table);
    *out = B;
    return RMHDLB_OK;
}

rmhdlb_ctx* rmhdlb_batch_instance(rmhdlb_batch* B, int32_t i) {
    return (B && i >= 0 && i < B->n) ? B->ctx[i] : nullptr;
}

int rmhdlb_batch_destroy(rmhdlb_batch* B) {
    if (!B) return RMHDLB_OK;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    drop_graphs(B);
    for (rmhdlb_ctx* C : B->ctx) rmhdlb_destroy(C);
    if (B->dev) (void)hipFree(B->dev);
    delete B;
    return RMHDLB_OK;
}

int rmhdlb_batch_step(rmhdlb_batch* B, int64_t nsteps) {
    if (!B || nsteps < 0) return RMHDLB_EINVAL;
    int rc = check_batch_state(B);
    if (rc != RMHDLB_OK) return rc;
    if (nsteps == 0) return RMHDLB_OK;
    rc = batch_table(B);
    if (rc != RMHDLB_OK) return rc;
    // an instance's tuning or the batch's shape may have changed the grid since the capture
    if (!(batch_geom(B) == B->graph_geom)) {
        drop_graphs(B);
        B->graph_geom = batch_geom(B);
    }
    int parity = B->ctx[0]->cur;
    if (B->persistent && B->total_face > 0) return RMHDLB_EUNSUPPORTED;  // no face pass in the persistent kernel
    if (B->persistent) {
        for (int64_t done = 0; done < nsteps;) {
            const int chunk = (int)std::min<int64_t>(nsteps - done, 1 << 30);
            if (batch_launch_persistent(B, parity, chunk) != hipSuccess) return RMHDLB_EDEVICE;
            parity = (parity + chunk) & 1;
            done += chunk;
        }
        for (rmhdlb_ctx* C : B->ctx) {
            C->cur = parity;
            C->step += nsteps;
        }
        return RMHDLB_OK;
    }
    int64_t left = nsteps;
    if (parity == 1) {
        if (batch_launch(B, 1) != hipSuccess) return RMHDLB_EDEVICE;
        parity = 0;
        --left;
    }
    if (left >= GRAPH_LONG && !B->exec_long) B->exec_long = capture_steps(B, GRAPH_LONG);
    while (left >= GRAPH_LONG && B->exec_long) {
        if (hipGraphLaunch(B->exec_long, B->stream) != hipSuccess) return RMHDLB_EDEVICE;
        left -= GRAPH_LONG;
    }
    if (left >= 2 && !B->exec_pair) B->exec_pair = capture_steps(B, 2);
    while (left >= 2) {
        if (B->exec_pair) {
            if (hipGraphLaunch(B->exec_pair, B->stream) != hipSuccess) return RMHDLB_EDEVICE;
        } else if (batch_launch(B, 0) != hipSuccess || batch_launch(B, 1) != hipSuccess) {
            return RMHDLB_EDEVICE;
        }
        left -= 2;
    }
    if (left == 1) {
        if (batch_launch(B, 0) != hipSuccess) return RMHDLB_EDEVICE;
        parity = 1;
    }
    for (rmhdlb_ctx* C : B->ctx) {
        C->cur = parity;
        C->step += nsteps;
    }
    return RMHDLB_OK;
}

int rmhdlb_batch_set_persistent(rmhdlb_batch* B, int32_t on) {
    if (!B || (on != 0 && on != 1)) return RMHDLB_EINVAL;
    if (on) {
        int dev = 0, coop = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess)
            return RMHDLB_EDEVICE;
        if (!coop) return RMHDLB_EUNSUPPORTED;
    }
    B->persistent = on;
    return RMHDLB_OK;
}

int rmhdlb_batch_set_tuning(rmhdlb_batch* B, int32_t px, int32_t yw, int32_t waves) {
    if (!B || (px != 128 && px != 64 && px != 32 && px != 16) || yw < 1 || yw > 8 || (waves != 2 && waves != 3))
        return RMHDLB_EINVAL;
    if (waves == 3 && B->storage != RMHDLB_STORE_F32) return RMHDLB_EINVAL;
    B->px = px;
    B->yw = yw;
    B->waves = waves;
    return RMHDLB_OK;
}

int rmhdlb_batch_autotune(rmhdlb_batch* B, int32_t* px_out, int32_t* yw_out, int32_t* waves_out) {
    if (!B) return RMHDLB_EINVAL;
    int rc = check_batch_state(B);
    if (rc != RMHDLB_OK) return rc;
    const int parity = B->ctx[0]->cur;
    BatchKey key;
    key.first = B->storage;
    for (rmhdlb_ctx* C : B->ctx) key.second.emplace_back(C->K.nx, C->K.ny, C->K.nz);
    BatchShape best{64, 1, 2};
    bool cached = false;
    {
        std::lock_guard<std::mutex> g(g_tune_mutex);
        auto it = g_batch_cache.find(key);
        if (it != g_batch_cache.end()) {
            best = it->second;
            cached = true;
        }
    }
    if (!cached) {
        // tiles px x (cells per row group / px) yw, times the occupancy variants of the storage type:
        // pair layout (FP64: 128 cells) 64x2, 32x4, 16x8, 64x4, 32x8, 128x2, 16x16, 64x8; quad and
        // double-quad layouts (FP32, FP16: 256 cells) 64x4, 32x8, 16x16, 128x2, 64x8, 32x16, 128x4, 16x32
        const BatchShape pair_shapes[8] = {{64, 1, 0}, {32, 1, 0}, {16, 1, 0}, {64, 2, 0},
                                           {32, 2, 0}, {128, 2, 0}, {16, 2, 0}, {64, 4, 0}};
        const BatchShape quad_shapes[8] = {{64, 1, 0}, {32, 1, 0}, {16, 1, 0}, {128, 1, 0},
                                           {64, 2, 0}, {32, 2, 0}, {128, 2, 0}, {16, 2, 0}};
        const BatchShape* shapes = rmhd::quad_storage(B->storage) ? quad_shapes : pair_shapes;
        float best_ms = 1e30f;
        for (int si = 0; si < 8; ++si)
            for (int waves : {2, 3}) {
                const BatchShape& sh = shapes[si];
                if (waves == 3 && B->storage != RMHDLB_STORE_F32) continue;
                B->px = sh.px;
                B->yw = sh.yw;
                B->waves = waves;
                rc = batch_table(B);
                if (rc != RMHDLB_OK) return rc;
                float ms = 0.0f;
                rc = time_ms(B->stream, 3, [&]() { return batch_launch(B, parity); }, &ms);
                if (rc != RMHDLB_OK) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = BatchShape{sh.px, sh.yw, waves};
                }
            }
        std::lock_guard<std::mutex> g(g_tune_mutex);
        g_batch_cache[key] = best;
    }
    B->px = best.px;
    B->yw = best.yw;
    B->waves = best.waves;
    if (px_out) *px_out = best.px;
    if (yw_out) *yw_out = best.yw;
    if (waves_out) *waves_out = best.waves;
    return RMHDLB_OK;
}

int64_t rmhdlb_state_len(const rmhdlb_ctx* C) { return C ? (int64_t)rmhd::state_arrays(C->K) * C->K.N : -1; }

int rmhdlb_get_state(rmhdlb_ctx* C, double* dst) {
    if (!C || !dst) return RMHDLB_EINVAL;
    if (!C->has_state) return RMHDLB_ESTATE;
    hipError_t e = RMHD_DISPATCH(C, launch_export)(C->sb[C->cur], dst, C->K, C->stream);
    if (e != hipSuccess || hipStreamSynchronize(C->stream) != hipSuccess) return RMHDLB_EDEVICE;
    return RMHDLB_OK;
}

int rmhdlb_set_state(rmhdlb_ctx* C, const double* src) {
    if (!C || !src) return RMHDLB_EINVAL;
    hipError_t e = RMHD_DISPATCH(C, launch_import)(src, C->sb[C->cur], C->K, C->stream);
    if (e != hipSuccess || hipStreamSynchronize(C->stream) != hipSuccess) return RMHDLB_EDEVICE;
    C->has_state = true;
    return C->guess_mode == RMHDLB_GUESS_MLP ? arm_gate(C, false) : RMHDLB_OK;
}

int rmhdlb_lattice_tables(int32_t* e19, double* w19, int32_t* s24, int32_t* ehat24, int32_t* bhat24) {
    if (!e19 || !w19 || !s24 || !ehat24 || !bhat24) return RMHDLB_EINVAL;
    for (int i = 0; i < rmhd::Q; ++i) {
        e19[3 * i] = rmhd::EX[i];
        e19[3 * i + 1] = rmhd::EY[i];
        e19[3 * i + 2] = rmhd::EZ[i];
        w19[i] = rmhd::weight(i);
    }
    for (int k = 0; k < rmhd::QH; ++k) {
        s24[3 * k] = rmhd::SX[k];
        s24[3 * k + 1] = rmhd::SY[k];
        s24[3 * k + 2] = rmhd::SZ[k];
        ehat24[3 * k] = rmhd::EHX[k];
        ehat24[3 * k + 1] = rmhd::EHY[k];
        ehat24[3 * k + 2] = rmhd::EHZ[k];
        bhat24[3 * k] = rmhd::BHX[k];
        bhat24[3 * k + 1] = rmhd::BHY[k];
        bhat24[3 * k + 2] = rmhd::BHZ[k];
    }
    return RMHDLB_OK;
}

}  // extern "C"
