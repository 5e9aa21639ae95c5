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

Layout sc_layout(const lbm_sc_params* p);
void sc_default_kernel(int Q, int nx, int ny, int nz, int* tx, int* ty, int* mb);
sc::StepParams sc_step_params(const lbm_sc* h, int parity);
hipError_t sc_launch_step(lbm_sc* h, int parity, hipStream_t s);
int sc_enqueue_steps(lbm_sc* h, long long n, hipStream_t s);
