// sc_runtime.hip -- host runtime and C ABI of the single-lattice Shan-Chen
// library: validation, device memory layout, kernel configuration, the step
// loop (with HIP graph replay for launch-bound lattices), observables and
// population transfer.  See include/lbm_sc.h for the contract.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/lbm_sc.h"
#include "sc_internal.h"
#include "sc_runtime.h"

using namespace sc;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

thread_local char g_last_error[256] = "";

void note_hip(hipError_t e, const char* where) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
}

int validate(const lbm_sc_params* p) {
    if (!p) return LBM_EINVAL;
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return LBM_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBM_EINVAL;
    if (p->lattice == LBM_D2Q9 && p->nz != 1) return LBM_EINVAL;
    const unsigned long long n = (unsigned long long)p->nx * p->ny * p->nz;
    if (n >= (1ull << 29)) return LBM_EINVAL;
    // every population array, padding included, within 32-bit byte offsets
    if ((unsigned long long)sc_array_stride(p) * 8ull > 0xFFFFFFFFull) return LBM_EINVAL;
    if (!(p->tau_A > 0.5) || !(p->tau_B > 0.5) || !isfinite(p->tau_A) || !isfinite(p->tau_B))
        return LBM_EINVAL;
    if (!(p->G >= 0.0) || !isfinite(p->G)) return LBM_EINVAL;
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32_SHIFTED) return LBM_EINVAL;
    if (!isfinite(p->body_A) || !isfinite(p->rho_ref_A) || !isfinite(p->rho_ref_B)) return LBM_EINVAL;
    if (p->forcing != LBM_FORCING_SHIFT && p->forcing != LBM_FORCING_GUO) return LBM_EINVAL;
    for (double tm : {p->tau_minus_A, p->tau_minus_B})
        if (!isfinite(tm) || (tm > 0.0 && !(tm > 0.5))) return LBM_EINVAL;
    return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Memory layout of one handle (all regions 256-byte aligned):
//   f0, f1   : population ping-pong buffers, 2 Q NS elements each (rows px apart)
//   psi      : two-pass density array, 2 N arithmetic elements
//   rho      : FP64 densities 2 N (observables; init staging)
//   u        : FP64 velocity 3 N (observables; init staging; population staging)
//   partial  : observables block partials
//   totals   : T_COUNT doubles
// ---------------------------------------------------------------------------
// Elements from one population array to the next.  N is rounded up to 32
// elements so that every array starts 256-byte (FP64) / 128-byte (FP32)
// aligned, like the first, and lattices of 2^16 sites or more get 2080 more
// elements (16.25 KB FP64, 8.1 KB FP32): with a stride of exactly N = 2^k
// sites the 2Q arrays start at the same offset modulo a large power of two
// and the step's 4Q concurrent streams contend for the same HBM channels and
// banks.  Measured on the 256^3 D3Q19 step: FP64 2.31-2.35 -> 2.25 ms, FP32
// 1.062 -> 1.010 ms; an unaligned stride (N + 37) ran at 2.66 / 1.52 ms.
// Smaller lattices are cache resident and keep the plain rounded stride.
constexpr size_t kArrayPad = 2080;
constexpr size_t kArrayPadMinSites = size_t(1) << 16;

namespace {

size_t padded_stride(size_t elems, size_t sites) {
    return (elems + 31) / 32 * 32 + (sites >= kArrayPadMinSites ? kArrayPad : 0);
}

}  // namespace

// Elements from one x row of a population array to the next.  Lattices of
// 2^16 sites or more round it up to 32 elements, so that every row starts
// 128-byte (FP32) / 256-byte (FP64) aligned like the arrays: with rows of nx
// elements a wave's 64 consecutive sites straddle one more cache line and
// its stores write partial lines.  Measured on D3Q19 FP32 steps with the
// plain row: 200^3 10,560, 216^3 11,120, 249^3 9,460 MLUPS, against 15,140
// at 192^3 and 16,580 at 256^3 (rows of 768 and 1024 bytes).  The padding
// columns are never written or read.  The row stays nx elements where the
// padded arrays would leave 32-bit byte offsets.
uint32_t sc_row_pitch(const lbm_sc_params* p) {
    const size_t nx = (size_t)p->nx, rows = (size_t)p->ny * p->nz, N = nx * rows;
    if (N < kArrayPadMinSites || nx % 32 == 0) return (uint32_t)nx;
    const size_t px = (nx + 31) / 32 * 32;
    if (padded_stride(px * rows, N) * 8 > 0xFFFFFFFFull) return (uint32_t)nx;
    return (uint32_t)px;
}

uint32_t sc_array_stride(const lbm_sc_params* p) {
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    return (uint32_t)padded_stride((size_t)sc_row_pitch(p) * p->ny * p->nz, N);
}

Layout sc_layout(const lbm_sc_params* p) {
    Layout L{};
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t NS = sc_array_stride(p);
    const size_t es = p->precision == LBM_FP64 ? 8 : 4;
    size_t off = 0;
    L.f[0] = off;
    off += align_up(2 * (size_t)p->lattice * NS * es);
    L.f[1] = off;
    off += align_up(2 * (size_t)p->lattice * NS * es);
    L.psi = off;
    off += align_up(2 * N * es);
    L.rho = off;
    off += align_up(2 * N * 8);
    L.u = off;
    off += align_up(3 * N * 8);
    L.partial = off;
    off += align_up((size_t)observe_blocks((uint32_t)N) * T_COUNT * 8);
    L.totals = off;
    off += align_up(T_COUNT * 8);
    L.total = off;
    return L;
}

// Default kernel configuration: tile width close to the x extent, march chunk
// sized for about four waves of blocks on 256 CUs (at least 8 planes so the two
// extra density planes per chunk stay a small overhead).
// Kernel configuration of a new handle, the choice the autotuner made for the
// tuned lattices.  D2Q9: the fused march on a row tile of up to 256 sites,
// march chunks giving about 1024 blocks.  D3Q19: 64 x 8 tiles (32 x 4 for
// nx <= 32), the fused march in FP64 and the pipelined one in FP32 shifted
// (whose three register planes fit at two waves per SIMD), march chunks giving
// about one block per CU (256); at 128^3 and 256^3 this is exactly the tuned
// configuration of both precisions.
void sc_default_kernel(const lbm_sc_params* p, int* variant, int* tx, int* ty, int* mb) {
    const int Q = p->lattice, nx = p->nx, ny = p->ny, nz = p->nz;
    if (Q == 9) {
        *variant = 0;
        *tx = nx <= 64 ? 64 : (nx <= 128 ? 128 : 256);
        *ty = 1;
        const int ntx = (nx + *tx - 1) / *tx;
        const int NM = ny;
        int chunks = std::max(1, 1024 / ntx);
        int m = (NM + chunks - 1) / chunks;
        *mb = std::max(std::min(m, NM), std::min(8, NM));
    } else {
        const bool small = nx <= 32;
        *variant = p->precision == LBM_FP32_SHIFTED ? 2 : 0;
        *tx = small ? 32 : 64;
        *ty = small ? 4 : 8;
        const int tiles = ((nx + *tx - 1) / *tx) * ((ny + *ty - 1) / *ty);
        const int NM = nz;
        int chunks = std::max(1, 256 / tiles);
        int m = (NM + chunks - 1) / chunks;
        *mb = std::max(std::min(m, NM), std::min(8, NM));
    }
}

StepParams sc_step_params(const lbm_sc* h, int parity) {
    StepParams sp{};
    const lbm_sc_params& p = h->p;
    sp.src = h->f[parity];
    sp.dst = h->f[parity ^ 1];
    if (h->Q == 19) {
        sp.NX = p.nx;
        sp.NY = p.ny;
        sp.NM = p.nz;
    } else {
        sp.NX = p.nx;
        sp.NY = 1;
        sp.NM = p.ny;
    }
    sp.PX = h->PX;
    sp.P = (uint32_t)sp.PX * (uint32_t)sp.NY;
    sp.N = h->N;
    sp.NS = h->NS;
    sp.ntx = (sp.NX + h->tx - 1) / h->tx;
    sp.nty = (sp.NY + h->ty - 1) / h->ty;
    sp.mb = std::max(1, std::min(h->mb, sp.NM));
    sp.nchunks = (sp.NM + sp.mb - 1) / sp.mb;
    sp.ny_lat = p.ny;
    sp.tau[0] = p.tau_A;
    sp.tau[1] = p.tau_B;
    sp.omega[0] = 1.0 / p.tau_A;
    sp.omega[1] = 1.0 / p.tau_B;
    for (int s = 0; s < 2; ++s) {
        sp.tau_m[s] = sc_tau_minus(p, s);
        sp.omega_m[s] = 1.0 / sp.tau_m[s];
    }
    sp.G = p.G;
    sp.rho_ref[0] = h->rho_ref[0];
    sp.rho_ref[1] = h->rho_ref[1];
    sp.body_A = p.body_A;
    sp.forcing = p.forcing;
    return sp;
}

hipError_t sc_launch_step(lbm_sc* h, int parity, hipStream_t s) {
    const StepParams sp = sc_step_params(h, parity);
    return launch_step(h->variant, h->Q, sc_policy(h->p), h->tx, h->ty, sp, h->psi, s);
}

namespace {

#define CHECK_H(h)                                            \
    do {                                                      \
        if (!(h)) return LBM_EINVAL;                          \
        if ((h)->err) return (h)->err;                        \
    } while (0)

#define HIPCALL(h, expr)                                      \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) {                               \
            note_hip(e_, #expr);                              \
            (h)->err = LBM_EDEVICE;                           \
            return LBM_EDEVICE;                               \
        }                                                     \
    } while (0)

void drop_graphs(lbm_sc* h) {
    for (int k = 0; k < 2; ++k) {
        if (h->gexec[k]) (void)hipGraphExecDestroy(h->gexec[k]);
        h->gexec[k] = nullptr;
    }
}

// Graph replay pays when a step is short compared with a launch: lattices
// whose population traffic per step is below 256 MB.
bool wants_graph(const lbm_sc* h) {
    const double bytes = 4.0 * h->Q * (double)h->N * (h->p.precision == LBM_FP64 ? 8 : 4);
    return bytes < 256.0 * 1024 * 1024;
}

int capture_graph(lbm_sc* h, int parity) {
    hipGraph_t g = nullptr;
    HIPCALL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int par = parity;
    hipError_t le = hipSuccess;
    for (int k = 0; k < kGraphSteps && le == hipSuccess; ++k) {
        le = sc_launch_step(h, par, h->stream);
        par ^= 1;
    }
    hipError_t ee = hipStreamEndCapture(h->stream, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        note_hip(le != hipSuccess ? le : ee, "graph capture");
        h->err = LBM_EDEVICE;
        return LBM_EDEVICE;
    }
    hipError_t ie = hipGraphInstantiate(&h->gexec[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        note_hip(ie, "hipGraphInstantiate");
        h->gexec[parity] = nullptr;
        h->err = LBM_EDEVICE;
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

}  // namespace

int sc_enqueue_steps(lbm_sc* h, long long n, hipStream_t s, bool allow_graph) {
    if (n <= 0) return LBM_OK;
    if (allow_graph && s == h->stream && n >= kGraphSteps && wants_graph(h)) {
        while (n >= kGraphSteps) {
            if (!h->gexec[h->cur]) {
                int rc = capture_graph(h, h->cur);
                if (rc) return rc;
            }
            HIPCALL(h, hipGraphLaunch(h->gexec[h->cur], h->stream));
            n -= kGraphSteps;
            h->steps += kGraphSteps;  // even count: parity unchanged
        }
    }
    for (long long k = 0; k < n; ++k) {
        HIPCALL(h, sc_launch_step(h, h->cur, s));
        h->cur ^= 1;
        h->steps += 1;
    }
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int lbm_sc_params_default(lbm_sc_params* p, int lattice, int nx, int ny, int nz, double tau_A,
                          double tau_B, double G) {
    if (!p) return LBM_EINVAL;
    memset(p, 0, sizeof(*p));
    p->lattice = lattice;
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->tau_A = tau_A;
    p->tau_B = tau_B;
    p->G = G;
    p->precision = LBM_FP64;
    p->rho_ref_A = 0.0;
    p->rho_ref_B = 0.0;
    p->body_A = 0.0;
    p->forcing = LBM_FORCING_SHIFT;
    p->tau_minus_A = p->tau_minus_B = 0.0;
    return validate(p);
}

size_t lbm_sc_bytes_needed(const lbm_sc_params* p) {
    if (validate(p) != LBM_OK) return 0;
    return sc_layout(p).total;
}

int lbm_sc_create(lbm_sc** out, int lattice, int nx, int ny, int nz, double tau_A, double tau_B,
                  double G) {
    lbm_sc_params p;
    int rc = lbm_sc_params_default(&p, lattice, nx, ny, nz, tau_A, tau_B, G);
    if (rc) return rc;
    return lbm_sc_create_ex(out, &p, nullptr, nullptr, 0);
}

int lbm_sc_create_ex(lbm_sc** out, const lbm_sc_params* p, void* stream, void* arena,
                     size_t arena_bytes) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    const Layout L = sc_layout(p);
    if (arena && (arena_bytes < L.total || ((uintptr_t)arena % kAlign) != 0)) return LBM_ENOMEM;
    lbm_sc* h = new (std::nothrow) lbm_sc();
    if (!h) return LBM_ENOMEM;
    h->p = *p;
    h->Q = p->lattice;
    h->N = (uint32_t)((size_t)p->nx * p->ny * p->nz);
    h->NS = sc_array_stride(p);
    h->PX = (int)sc_row_pitch(p);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        note_hip(e, "hipGetDevice");
        delete h;
        return LBM_EDEVICE;
    }
    if (arena) {
        h->mem = static_cast<char*>(arena);
        h->own_mem = false;
    } else {
        void* m = nullptr;
        e = hipMalloc(&m, L.total);
        if (e != hipSuccess) {
            note_hip(e, "hipMalloc");
            delete h;
            return LBM_ENOMEM;
        }
        h->mem = static_cast<char*>(m);
        h->own_mem = true;
    }
    h->mem_bytes = L.total;
    h->layout = L;
    h->f[0] = h->mem + L.f[0];
    h->f[1] = h->mem + L.f[1];
    h->psi = h->mem + L.psi;
    h->rho = reinterpret_cast<double*>(h->mem + L.rho);
    h->u = reinterpret_cast<double*>(h->mem + L.u);
    h->partial = reinterpret_cast<double*>(h->mem + L.partial);
    h->totals = reinterpret_cast<double*>(h->mem + L.totals);
    if (stream) {
        h->stream = static_cast<hipStream_t>(stream);
        h->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            note_hip(e, "hipStreamCreate");
            if (h->own_mem) (void)hipFree(h->mem);
            delete h;
            return LBM_EDEVICE;
        }
        h->own_stream = true;
    }
    if (hipEventCreate(&h->ev[0]) != hipSuccess || hipEventCreate(&h->ev[1]) != hipSuccess) {
        note_hip(hipErrorUnknown, "hipEventCreate");
        if (h->own_stream) (void)hipStreamDestroy(h->stream);
        if (h->own_mem) (void)hipFree(h->mem);
        delete h;
        return LBM_EDEVICE;
    }
    sc_default_kernel(p, &h->variant, &h->tx, &h->ty, &h->mb);
    h->rho_ref[0] = p->rho_ref_A;
    h->rho_ref[1] = p->rho_ref_B;
    *out = h;
    return LBM_OK;
}

int lbm_sc_init(lbm_sc* h, const double* rho_A, const double* rho_B, const double* u) {
    CHECK_H(h);
    if (!rho_A || !rho_B) return LBM_EINVAL;
    if (h->batch) return LBM_ESTATE;
    const size_t N = h->N;
    double sum[2] = {0.0, 0.0};
    for (size_t x = 0; x < N; ++x) {
        if (!(rho_A[x] > 0.0) || !(rho_B[x] > 0.0) || !isfinite(rho_A[x]) || !isfinite(rho_B[x]))
            return LBM_EINVAL;
        sum[0] += rho_A[x];
        sum[1] += rho_B[x];
    }
    if (u)
        for (size_t k = 0; k < 3 * N; ++k)
            if (!isfinite(u[k])) return LBM_EINVAL;
    if (h->p.precision == LBM_FP32_SHIFTED) {
        h->rho_ref[0] = h->p.rho_ref_A > 0.0 ? h->p.rho_ref_A : sum[0] / (double)N;
        h->rho_ref[1] = h->p.rho_ref_B > 0.0 ? h->p.rho_ref_B : sum[1] / (double)N;
    } else {
        h->rho_ref[0] = h->rho_ref[1] = 0.0;
    }
    drop_graphs(h);  // the reference densities are baked into captured launches
    (void)hipSetDevice(h->device);
    HIPCALL(h, hipMemcpyAsync(h->rho, rho_A, N * 8, hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->rho + N, rho_B, N * 8, hipMemcpyHostToDevice, h->stream));
    if (u) HIPCALL(h, hipMemcpyAsync(h->u, u, 3 * N * 8, hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, launch_init(h->Q, h->p.precision, h->f[0], h->NS, h->rho, u ? h->u : nullptr, h->p.nx,
                           h->p.ny, h->p.nz, h->PX, h->rho_ref, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    h->cur = 0;
    h->steps = 0;
    h->inited = true;
    return LBM_OK;
}

int lbm_sc_step(lbm_sc* h, int n) {
    CHECK_H(h);
    if (n < 0) return LBM_EINVAL;
    if (!h->inited) return LBM_ESTATE;
    if (h->batch) return LBM_ESTATE;
    (void)hipSetDevice(h->device);
    return sc_enqueue_steps(h, n, h->stream);
}

int lbm_sc_set_probe(lbm_sc* h, double cx, double cy, double cz, double R) {
    CHECK_H(h);
    if (!isfinite(cx) || !isfinite(cy) || !isfinite(cz) || !isfinite(R)) return LBM_EINVAL;
    if (R <= 0.0) {
        h->has_probe = false;
        return LBM_OK;
    }
    h->has_probe = true;
    h->probe[0] = cx;
    h->probe[1] = cy;
    h->probe[2] = cz;
    h->probe[3] = R;
    return LBM_OK;
}

int lbm_sc_moments(lbm_sc* h, double* rho_A, double* rho_B, double* u, lbm_sc_totals* t) {
    CHECK_H(h);
    if (!h->inited) return LBM_ESTATE;
    (void)hipSetDevice(h->device);
    const size_t N = h->N;
    ObsArgs a{};
    a.f = h->f[h->cur];
    a.rho = h->rho;
    a.u = h->u;
    a.partial = h->partial;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.px = h->PX;
    a.N = h->N;
    a.NS = h->NS;
    a.G = h->p.G;
    a.body_A = h->p.body_A;
    a.rho_ref[0] = h->rho_ref[0];
    a.rho_ref[1] = h->rho_ref[1];
    a.has_probe = h->has_probe ? 1 : 0;
    for (int k = 0; k < 4; ++k) a.probe[k] = h->probe[k];
    if (h->has_probe) {
        const double R = h->probe[3];
        double half = 0.5 * std::min(h->p.nx, h->p.ny);
        if (h->p.nz > 1) half = std::min(half, 0.5 * h->p.nz);
        a.r_in = std::max(1.0, R / 4.0);
        a.r_out = R + 0.5 * (half - R);
    }
    HIPCALL(h, launch_observe(h->Q, h->p.precision, a, h->totals, h->stream));
    double T[T_COUNT];
    HIPCALL(h, hipMemcpyAsync(T, h->totals, sizeof(T), hipMemcpyDeviceToHost, h->stream));
    if (rho_A) HIPCALL(h, hipMemcpyAsync(rho_A, h->rho, N * 8, hipMemcpyDeviceToHost, h->stream));
    if (rho_B)
        HIPCALL(h, hipMemcpyAsync(rho_B, h->rho + N, N * 8, hipMemcpyDeviceToHost, h->stream));
    if (u) HIPCALL(h, hipMemcpyAsync(u, h->u, 3 * N * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    if (t) {
        memset(t, 0, sizeof(*t));
        t->mass_A = T[T_MASS_A];
        t->mass_B = T[T_MASS_B];
        t->mom[0] = T[T_MOM_X];
        t->mom[1] = T[T_MOM_Y];
        t->mom[2] = T[T_MOM_Z];
        t->max_u = T[T_MAX_U];
        t->ke = T[T_KE];
        t->n_in = T[T_N_IN];
        t->n_out = T[T_N_OUT];
        t->n_phi_pos = T[T_N_PHI_POS];
        t->n_nonfinite = T[T_N_NONFINITE];
        t->step = h->steps;
        if (h->has_probe && T[T_N_IN] > 0 && T[T_N_OUT] > 0) {
            t->p_in = T[T_P_IN] / T[T_N_IN];
            t->p_out = T[T_P_OUT] / T[T_N_OUT];
            t->rhoA_in = T[T_RA_IN] / T[T_N_IN];
            t->rhoA_out = T[T_RA_OUT] / T[T_N_OUT];
            t->dp = t->p_in - t->p_out;
            const int d = h->p.nz > 1 ? 3 : 2;
            const double cd = d == 3 ? 4.0 * M_PI / 3.0 : M_PI;
            const double num = t->mass_A - t->rhoA_out * (double)N;
            const double den = cd * (t->rhoA_in - t->rhoA_out);
            t->R_eff = pow(num / den, 1.0 / d);
        } else {
            t->p_in = t->p_out = t->dp = t->R_eff = NAN;
            t->rhoA_in = t->rhoA_out = NAN;
        }
    }
    const bool bad = T[T_N_NONFINITE] > 0 || !isfinite(T[T_MASS_A]) || !isfinite(T[T_MASS_B]) ||
                     !isfinite(T[T_MOM_X]) || !isfinite(T[T_MOM_Y]) || !isfinite(T[T_MOM_Z]);
    return bad ? LBM_ENONFINITE : LBM_OK;
}

int lbm_sc_get_populations(lbm_sc* h, double* f) {
    CHECK_H(h);
    if (!f) return LBM_EINVAL;
    if (!h->inited) return LBM_ESTATE;
    (void)hipSetDevice(h->device);
    const size_t N = h->N;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < h->Q; ++i) {
            HIPCALL(h, launch_get_plane(h->Q, h->p.precision, h->f[h->cur], h->NS, h->u, s, i, h->p.nx,
                                        h->p.ny, h->p.nz, h->PX, h->rho_ref, h->stream));
            HIPCALL(h, hipMemcpyAsync(f + ((size_t)s * h->Q + i) * N, h->u, N * 8,
                                      hipMemcpyDeviceToHost, h->stream));
            HIPCALL(h, hipStreamSynchronize(h->stream));
        }
    return LBM_OK;
}

int lbm_sc_set_populations(lbm_sc* h, const double* f) {
    CHECK_H(h);
    if (!f) return LBM_EINVAL;
    if (h->batch) return LBM_ESTATE;
    const size_t total = 2 * (size_t)h->Q * h->N;
    for (size_t k = 0; k < total; ++k)
        if (!isfinite(f[k])) return LBM_EINVAL;
    (void)hipSetDevice(h->device);
    const size_t N = h->N;
    if (h->p.precision == LBM_FP32_SHIFTED && !h->inited) {
        // reference densities from the given state: mean of sum_i f_is
        for (int s = 0; s < 2; ++s) {
            double acc = 0.0;
            for (int i = 0; i < h->Q; ++i)
                for (size_t x = 0; x < N; ++x) acc += f[((size_t)s * h->Q + i) * N + x];
            const double pr = s == 0 ? h->p.rho_ref_A : h->p.rho_ref_B;
            h->rho_ref[s] = pr > 0.0 ? pr : acc / (double)N;
        }
    }
    drop_graphs(h);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < h->Q; ++i) {
            HIPCALL(h, hipMemcpyAsync(h->u, f + ((size_t)s * h->Q + i) * N, N * 8,
                                      hipMemcpyHostToDevice, h->stream));
            HIPCALL(h, launch_set_plane(h->Q, h->p.precision, h->f[0], h->NS, h->u, s, i, h->p.nx,
                                        h->p.ny, h->p.nz, h->PX, h->rho_ref, h->stream));
        }
    HIPCALL(h, hipStreamSynchronize(h->stream));
    h->cur = 0;
    h->inited = true;
    return LBM_OK;
}

int lbm_sc_sync(lbm_sc* h) {
    CHECK_H(h);
    HIPCALL(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_sc_time_steps(lbm_sc* h, int n, float* ms) {
    CHECK_H(h);
    if (n < 0 || !ms) return LBM_EINVAL;
    if (!h->inited) return LBM_ESTATE;
    if (h->batch) return LBM_ESTATE;
    (void)hipSetDevice(h->device);
    HIPCALL(h, hipEventRecord(h->ev[0], h->stream));
    int rc = sc_enqueue_steps(h, n, h->stream);
    if (rc) return rc;
    HIPCALL(h, hipEventRecord(h->ev[1], h->stream));
    HIPCALL(h, hipEventSynchronize(h->ev[1]));
    HIPCALL(h, hipEventElapsedTime(ms, h->ev[0], h->ev[1]));
    return LBM_OK;
}

int lbm_sc_set_kernel(lbm_sc* h, int variant, int tx, int ty, int mb) {
    CHECK_H(h);
    if (variant < 0 || variant > 3) return LBM_EINVAL;
    if (h->Q == 9 && ty != 1) return LBM_EINVAL;
    if (!tile_supported(h->Q, tx, ty)) return LBM_EINVAL;
    if (mb < 1) return LBM_EINVAL;
    h->variant = variant;
    h->tx = tx;
    h->ty = ty;
    h->mb = mb;
    drop_graphs(h);
    return LBM_OK;
}

int lbm_sc_get_kernel(const lbm_sc* h, int* variant, int* tx, int* ty, int* mb) {
    if (!h) return LBM_EINVAL;
    if (variant) *variant = h->variant;
    if (tx) *tx = h->tx;
    if (ty) *ty = h->ty;
    if (mb) *mb = std::min(h->mb, h->Q == 19 ? h->p.nz : h->p.ny);
    return LBM_OK;
}

int lbm_sc_tile_count(int lattice) { return tile_count(lattice); }

int lbm_sc_tile_get(int lattice, int k, int* tx, int* ty) {
    if (!tx || !ty) return LBM_EINVAL;
    return tile_get(lattice, k, tx, ty) ? LBM_OK : LBM_EINVAL;
}

long long lbm_sc_steps_done(const lbm_sc* h) { return h ? h->steps : -1; }

int lbm_sc_get_params(const lbm_sc* h, lbm_sc_params* p) {
    if (!h || !p) return LBM_EINVAL;
    *p = h->p;
    if (h->p.precision == LBM_FP32_SHIFTED) {
        p->rho_ref_A = h->rho_ref[0];
        p->rho_ref_B = h->rho_ref[1];
    }
    return LBM_OK;
}

int lbm_sc_device_buffers(const lbm_sc* h, void** buf0, void** buf1, int* current) {
    if (!h) return LBM_EINVAL;
    if (buf0) *buf0 = h->f[0];
    if (buf1) *buf1 = h->f[1];
    if (current) *current = h->cur;
    return LBM_OK;
}

int lbm_sc_buffer_layout(const lbm_sc* h, size_t* stride, int* pitch) {
    if (!h) return LBM_EINVAL;
    if (stride) *stride = h->NS;
    if (pitch) *pitch = h->PX;
    return LBM_OK;
}

int lbm_sc_destroy(lbm_sc* h) {
    if (!h) return LBM_OK;
    if (h->batch) return LBM_ESTATE;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    (void)hipEventDestroy(h->ev[0]);
    (void)hipEventDestroy(h->ev[1]);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    if (h->own_mem) (void)hipFree(h->mem);
    delete h;
    return LBM_OK;
}

const char* lbm_sc_strerror(int status) {
    switch (status) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "out of device memory or arena too small";
        case LBM_EDEVICE: return g_last_error[0] ? g_last_error : "HIP runtime error";
        case LBM_ESTATE: return "call out of order for this handle";
        case LBM_ENONFINITE: return "non-finite density or velocity";
        case LBM_EBUDGET: return "batch memory budget exceeded";
        case LBM_ETIMEOUT: return "persistent launch hit its grid-barrier spin limit";
        case LBM_ETOOBIG:
            return "batch group exceeds the allocation-free scratch (1024 members, 262144 work items)";
        default: return "unknown status";
    }
}

int lbm_sc_copy_bench(void* dst, const void* src, size_t nbytes, int reps, void* stream,
                      float* ms) {
    if (!dst || !src || !ms || reps < 1 || nbytes < 8) return LBM_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_EDEVICE;
    }
    hipError_t e = launch_copy(dst, src, nbytes, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(dst, src, nbytes, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        note_hip(e, "copy bench");
        return LBM_EDEVICE;
    }
    *ms = t / reps;
    return LBM_OK;
}

}  // extern "C"
