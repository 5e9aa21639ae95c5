// sc_steps.h -- the single-lattice step kernels, templated on the policy
// (storage precision, forcing scheme, relaxation), with their host
// launchers.  Each policy is instantiated in a translation unit of its own
// (sc_step_<policy>.hip), so that the policies compile in parallel and no
// policy carries another's code; the runtime reaches them through
// step_launch<P>.  The batch kernels are in sc_batch_kernels.h.
#pragma once

#include <hip/hip_runtime.h>

#include "sc_internal.h"

namespace sc {

// ---------------------------------------------------------------------------
// Fused step: one block per (tile, march chunk).
// ---------------------------------------------------------------------------
// Minimum waves per SIMD the register allocator must allow for the fused
// step: two planes of populations stay in registers without scratch at
// 2 waves (D3Q19 FP64, 218 VGPRs), 3 (D2Q9 FP64, D3Q19 FP32) and 4 (D2Q9 FP32).
template <int Q, class PR>
struct FusedWaves {
    static constexpr int value = PR::shifted ? (Q == 19 ? 3 : 4) : (Q == 19 ? 2 : 3);
};

template <int Q, class PR, int TX, int TY>
__global__ void __launch_bounds__(TX* TY)
    __attribute__((amdgpu_waves_per_eu(FusedWaves<Q, PR>::value))) k_step_fused(StepParams p) {
    using TS = TileStep<Q, PR, TX, TY>;
    __shared__ typename PR::A lds[TS::LDS_ELEMS];
    const int w = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tiles = p.ntx * p.nty;
    const int chunk = w / tiles;
    const int t = w - chunk * tiles;
    TS::run(p, t % p.ntx, t / p.ntx, chunk, lds);
}

template <int Q, class PR, int TX, int TY>
static hipError_t launch_fused_t(const StepParams& p, hipStream_t s) {
    const unsigned nblk = (unsigned)p.ntx * p.nty * p.nchunks;
    hipLaunchKernelGGL((k_step_fused<Q, PR, TX, TY>), dim3(nblk), dim3(TX * TY), 0, s, p);
    return hipGetLastError();
}

template <class PR>
static hipError_t launch_fused_p(int Q, int tx, int ty, const StepParams& p, hipStream_t s) {
    if (Q == 9) {
        switch (tx) {
            case 64: return launch_fused_t<9, PR, 64, 1>(p, s);
            case 128: return launch_fused_t<9, PR, 128, 1>(p, s);
            case 256: return launch_fused_t<9, PR, 256, 1>(p, s);
            case 512: return launch_fused_t<9, PR, 512, 1>(p, s);
        }
    } else {
        const int key = tx * 1000 + ty;
        switch (key) {
            case 32004: return launch_fused_t<19, PR, 32, 4>(p, s);
            case 64004: return launch_fused_t<19, PR, 64, 4>(p, s);
            case 32008: return launch_fused_t<19, PR, 32, 8>(p, s);
            case 64008: return launch_fused_t<19, PR, 64, 8>(p, s);
            case 16016: return launch_fused_t<19, PR, 16, 16>(p, s);
            case 32016: return launch_fused_t<19, PR, 32, 16>(p, s);
        }
    }
    return hipErrorInvalidValue;
}


// Pipelined march: three register planes; one wave per SIMD for D3Q19 FP64,
// two for D3Q19 FP32 and D2Q9 FP64, three for D2Q9 FP32.
template <int Q, class PR>
struct PipeWaves {
    static constexpr int value = PR::shifted ? (Q == 19 ? 2 : 3) : (Q == 19 ? 1 : 2);
};

template <int Q, class PR, int TX, int TY>
__global__ void __launch_bounds__(TX* TY)
    __attribute__((amdgpu_waves_per_eu(PipeWaves<Q, PR>::value))) k_step_pipe(StepParams p) {
    using TS = TileStepPipe<Q, PR, TX, TY>;
    __shared__ typename PR::A lds[TS::LDS_ELEMS];
    const int w = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tiles = p.ntx * p.nty;
    const int chunk = w / tiles;
    const int t = w - chunk * tiles;
    TS::run(p, t % p.ntx, t / p.ntx, chunk, lds);
}

template <int Q, class PR, int TX, int TY>
static hipError_t launch_pipe_t(const StepParams& p, hipStream_t s) {
    const unsigned nblk = (unsigned)p.ntx * p.nty * p.nchunks;
    hipLaunchKernelGGL((k_step_pipe<Q, PR, TX, TY>), dim3(nblk), dim3(TX * TY), 0, s, p);
    return hipGetLastError();
}

template <class PR>
static hipError_t launch_pipe_p(int Q, int tx, int ty, const StepParams& p, hipStream_t s) {
    if (Q == 9) {
        switch (tx) {
            case 64: return launch_pipe_t<9, PR, 64, 1>(p, s);
            case 128: return launch_pipe_t<9, PR, 128, 1>(p, s);
            case 256: return launch_pipe_t<9, PR, 256, 1>(p, s);
            case 512: return launch_pipe_t<9, PR, 512, 1>(p, s);
        }
    } else {
        const int key = tx * 1000 + ty;
        switch (key) {
            case 32004: return launch_pipe_t<19, PR, 32, 4>(p, s);
            case 64004: return launch_pipe_t<19, PR, 64, 4>(p, s);
            case 32008: return launch_pipe_t<19, PR, 32, 8>(p, s);
            case 64008: return launch_pipe_t<19, PR, 64, 8>(p, s);
            case 16016: return launch_pipe_t<19, PR, 16, 16>(p, s);
            case 32016: return launch_pipe_t<19, PR, 32, 16>(p, s);
        }
    }
    return hipErrorInvalidValue;
}



// Re-pull march: one register plane; three waves per SIMD for FP64, four for FP32.
template <int Q, class PR>
struct RepullWaves {
    // the Guo collision holds the force and its dot products: one wave less
    static constexpr int value = (PR::shifted ? 4 : 3) - (PR::guo ? 1 : 0);
};

template <int Q, class PR, int TX, int TY>
__global__ void __launch_bounds__(TX* TY)
    __attribute__((amdgpu_waves_per_eu(RepullWaves<Q, PR>::value))) k_step_repull(StepParams p) {
    using TS = TileStepRepull<Q, PR, TX, TY>;
    __shared__ typename PR::A lds[TS::LDS_ELEMS];
    const int w = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tiles = p.ntx * p.nty;
    const int chunk = w / tiles;
    const int t = w - chunk * tiles;
    TS::run(p, t % p.ntx, t / p.ntx, chunk, lds);
}

template <int Q, class PR, int TX, int TY>
static hipError_t launch_repull_t(const StepParams& p, hipStream_t s) {
    const unsigned nblk = (unsigned)p.ntx * p.nty * p.nchunks;
    hipLaunchKernelGGL((k_step_repull<Q, PR, TX, TY>), dim3(nblk), dim3(TX * TY), 0, s, p);
    return hipGetLastError();
}

template <class PR>
static hipError_t launch_repull_p(int Q, int tx, int ty, const StepParams& p, hipStream_t s) {
    if (Q == 9) {
        switch (tx) {
            case 64: return launch_repull_t<9, PR, 64, 1>(p, s);
            case 128: return launch_repull_t<9, PR, 128, 1>(p, s);
            case 256: return launch_repull_t<9, PR, 256, 1>(p, s);
            case 512: return launch_repull_t<9, PR, 512, 1>(p, s);
        }
    } else {
        const int key = tx * 1000 + ty;
        switch (key) {
            case 32004: return launch_repull_t<19, PR, 32, 4>(p, s);
            case 64004: return launch_repull_t<19, PR, 64, 4>(p, s);
            case 32008: return launch_repull_t<19, PR, 32, 8>(p, s);
            case 64008: return launch_repull_t<19, PR, 64, 8>(p, s);
            case 16016: return launch_repull_t<19, PR, 16, 16>(p, s);
            case 32016: return launch_repull_t<19, PR, 32, 16>(p, s);
        }
    }
    return hipErrorInvalidValue;
}


// ---------------------------------------------------------------------------
// Two-pass step: densities to an HBM psi array (one element per site, no row
// padding), then collide with a global gather.  Moves (6Q + 4) values per site instead of 4Q; kept as the plain
// form the fused kernel is measured against.
// ---------------------------------------------------------------------------
template <int Q, class PR>
__global__ void __launch_bounds__(256) k_density(StepParams p, typename PR::A* psi, int nx, int ny,
                                                 int nz) {
    using T = typename PR::T;
    using A = typename PR::A;
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= p.N) return;
    const T* f = static_cast<const T*>(p.src);
    const SiteGeom g = site_xyz(site, nx, ny);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        A r = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            r += A(f[(size_t)(s * Q + i) * p.NS +
                     elem_at(g, -VSet<Q>::cx(i), -VSet<Q>::cy(i), -VSet<Q>::cz(i), nx, ny, nz, p.PX)]);
        psi[(size_t)s * p.N + site] = r;
    }
}

template <int Q, class PR>
__global__ void __launch_bounds__(256) k_collide2(StepParams p, const typename PR::A* psi, int nx,
                                                  int ny, int nz) {
    using T = typename PR::T;
    using A = typename PR::A;
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= p.N) return;
    const T* f = static_cast<const T*>(p.src);
    const SiteGeom g = site_xyz(site, nx, ny);
    T v[2][Q];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i)
            v[s][i] = f[(size_t)(s * Q + i) * p.NS +
                        elem_at(g, -VSet<Q>::cx(i), -VSet<Q>::cy(i), -VSet<Q>::cz(i), nx, ny, nz, p.PX)];
    A gs[2][3];
    gather<Q>([&](int s, int i) {
        return psi[(size_t)s * p.N +
                   site_at(g, VSet<Q>::cx(i), VSet<Q>::cy(i), VSet<Q>::cz(i), nx, ny, nz)];
    }, gs);
    const double body = p.body_A != 0.0 ? kolmogorov(p, g.y) : 0.0;
    collide_store<Q, PR>(v, gs, p, body, static_cast<char*>(p.dst), p.NS * (uint32_t)sizeof(T),
                         elem_at(g, 0, 0, 0, nx, ny, nz, p.PX) * (uint32_t)sizeof(T), 0u);
}

template <int Q, class PR>
static hipError_t launch_twopass_t(const StepParams& p, void* psi, hipStream_t s) {
    using A = typename PR::A;
    const unsigned nblk = (p.N + 255u) / 256u;
    int nx, ny, nz;
    if (Q == 19) {
        nx = p.NX;
        ny = p.NY;
        nz = p.NM;
    } else {
        nx = p.NX;
        ny = p.NM;
        nz = 1;
    }
    hipLaunchKernelGGL((k_density<Q, PR>), dim3(nblk), dim3(256), 0, s, p, static_cast<A*>(psi),
                       nx, ny, nz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_collide2<Q, PR>), dim3(nblk), dim3(256), 0, s, p,
                       static_cast<const A*>(psi), nx, ny, nz);
    return hipGetLastError();
}


// Single-lattice step of one policy: variant 0 fused, 1 two-pass, 2 pipelined,
// 3 re-pull (psi is the two-pass density array).
template <class PR>
hipError_t step_launch(int variant, int Q, int tx, int ty, const StepParams& p, void* psi,
                       hipStream_t s) {
    switch (variant) {
        case 1:
            return Q == 9 ? launch_twopass_t<9, PR>(p, psi, s) : launch_twopass_t<19, PR>(p, psi, s);
        case 2: return launch_pipe_p<PR>(Q, tx, ty, p, s);
        case 3: return launch_repull_p<PR>(Q, tx, ty, p, s);
        default: return launch_fused_p<PR>(Q, tx, ty, p, s);
    }
}

#define SC_POLICIES(X) X(PF64) X(PF32S) X(PF64G) X(PF32SG) X(PF64T) X(PF32ST) X(PF64GT) X(PF32SGT)
#define SC_DECLARE(P)                                                                        \
    extern template hipError_t step_launch<P>(int, int, int, int, const StepParams&, void*, \
                                              hipStream_t);
SC_POLICIES(SC_DECLARE)
#undef SC_DECLARE

}  // namespace sc
