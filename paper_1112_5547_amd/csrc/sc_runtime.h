// sc_runtime.h -- internal definition of a lattice handle, shared by the
// single-lattice runtime and the batch engine (not exported).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm_sc.h"
#include "sc_internal.h"

struct Layout {
    size_t f[2], psi, rho, u, partial, totals, total;
};

// Steps per captured graph (even, so a replay leaves the parity unchanged).
constexpr int kGraphSteps = 32;

struct lbm_sc {
    lbm_sc_params p{};
    int Q = 0;
    uint32_t N = 0;
    uint32_t NS = 0;  // population array stride (elements), >= PX ny nz
    int PX = 0;       // population row pitch (elements), >= nx
    int device = 0;
    char* mem = nullptr;
    bool own_mem = false;
    size_t mem_bytes = 0;
    Layout layout{};
    void* f[2] = {nullptr, nullptr};
    int cur = 0;  // buffer holding the current state
    void* psi = nullptr;
    double* rho = nullptr;
    double* u = nullptr;
    double* partial = nullptr;
    double* totals = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int variant = 0, tx = 64, ty = 1, mb = 16;
    int err = 0;
    bool inited = false;
    double rho_ref[2] = {0.0, 0.0};
    bool has_probe = false;
    double probe[4] = {0, 0, 0, 0};
    long long steps = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    lbm_batch* batch = nullptr;  // batch this handle belongs to, if any
};

// Odd-part relaxation time of species s (tau_minus <= 0 means tau_s: BGK).
inline double sc_tau_minus(const lbm_sc_params& p, int s) {
    const double tm = s == 0 ? p.tau_minus_A : p.tau_minus_B;
    return tm > 0.0 ? tm : (s == 0 ? p.tau_A : p.tau_B);
}

// Kernel policy of a lattice (sc::step_policy index).
inline int sc_policy(const lbm_sc_params& p) {
    const bool trt = sc_tau_minus(p, 0) != p.tau_A || sc_tau_minus(p, 1) != p.tau_B;
    return sc::step_policy(p.precision, p.forcing, trt);
}

Layout sc_layout(const lbm_sc_params* p);
uint32_t sc_array_stride(const lbm_sc_params* p);
uint32_t sc_row_pitch(const lbm_sc_params* p);
void sc_default_kernel(const lbm_sc_params* p, int* variant, int* tx, int* ty, int* mb);
sc::StepParams sc_step_params(const lbm_sc* h, int parity);
hipError_t sc_launch_step(lbm_sc* h, int parity, hipStream_t s);
// Enqueues n steps on stream s.  allow_graph: replay captured 32-step graphs
// when s is the handle's own stream and the lattice is small enough for
// launches to dominate (the per-lattice batch baseline passes false: one
// launch per lattice per step, whichever stream it shares).
int sc_enqueue_steps(lbm_sc* h, long long n, hipStream_t s, bool allow_graph = true);
