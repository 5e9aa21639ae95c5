// sc_kernels.hip -- gfx950 kernels of the two-component Shan-Chen step and
// their host launchers: fused tile-march step, two-pass step, initial
// equilibrium, population export/import, FP64 observables with fixed-order
// reductions, and a streaming-copy bandwidth probe.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sc_batch_kernels.h"

namespace sc {

// ---------------------------------------------------------------------------
// Tile tables.  D2Q9 tiles are one x row (ty = 1); D3Q19 tiles are TX x TY.
// ---------------------------------------------------------------------------
struct TileShape {
    int tx, ty;
};
static const TileShape kTiles9[] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}};
static const TileShape kTiles19[] = {{32, 4}, {64, 4}, {32, 8}, {64, 8}, {16, 16}, {32, 16}};

int tile_count(int Q) {
    return Q == 9 ? (int)(sizeof(kTiles9) / sizeof(kTiles9[0]))
                  : (Q == 19 ? (int)(sizeof(kTiles19) / sizeof(kTiles19[0])) : 0);
}

bool tile_get(int Q, int k, int* tx, int* ty) {
    if (k < 0 || k >= tile_count(Q)) return false;
    const TileShape t = Q == 9 ? kTiles9[k] : kTiles19[k];
    *tx = t.tx;
    *ty = t.ty;
    return true;
}

bool tile_supported(int Q, int tx, int ty) {
    for (int k = 0; k < tile_count(Q); ++k) {
        int a, b;
        tile_get(Q, k, &a, &b);
        if (a == tx && b == ty) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Policy dispatch (the kernels are instantiated in sc_step_<policy>.hip).
// ---------------------------------------------------------------------------
hipError_t launch_step(int variant, int Q, int pol, int tx, int ty, const StepParams& p,
                       void* psi, hipStream_t s) {
    switch (pol) {
        case 0: return step_launch<PF64>(variant, Q, tx, ty, p, psi, s);
        case 1: return step_launch<PF32S>(variant, Q, tx, ty, p, psi, s);
        case 2: return step_launch<PF64G>(variant, Q, tx, ty, p, psi, s);
        case 3: return step_launch<PF32SG>(variant, Q, tx, ty, p, psi, s);
        case 4: return step_launch<PF64T>(variant, Q, tx, ty, p, psi, s);
        case 5: return step_launch<PF32ST>(variant, Q, tx, ty, p, psi, s);
        case 6: return step_launch<PF64GT>(variant, Q, tx, ty, p, psi, s);
        case 7: return step_launch<PF32SGT>(variant, Q, tx, ty, p, psi, s);
    }
    return hipErrorInvalidValue;
}

bool batch_kernels(int pol, int nt, int tx19, int ty19, BatchStepFn* sf, BatchPersFn* pf) {
    switch (pol) {
        case 0: return batch_fns<PF64>(nt, tx19, ty19, sf, pf);
        case 1: return batch_fns<PF32S>(nt, tx19, ty19, sf, pf);
        case 2: return batch_fns<PF64G>(nt, tx19, ty19, sf, pf);
        case 3: return batch_fns<PF32SG>(nt, tx19, ty19, sf, pf);
        case 4: return batch_fns<PF64T>(nt, tx19, ty19, sf, pf);
        case 5: return batch_fns<PF32ST>(nt, tx19, ty19, sf, pf);
        case 6: return batch_fns<PF64GT>(nt, tx19, ty19, sf, pf);
        case 7: return batch_fns<PF32SGT>(nt, tx19, ty19, sf, pf);
    }
    return false;
}

// ---------------------------------------------------------------------------
// Initial state: buf_is(y) = f_is^eq(rho_s(y + c_i), u(y + c_i)), so that the
// pulled read at x gives f_is(x, 0) = f^eq(rho_s(x), u(x)).
// ---------------------------------------------------------------------------
template <int Q, class PR>
__global__ void __launch_bounds__(256) k_init(typename PR::T* f, const double* rho, const double* u,
                                              int nx, int ny, int nz, int px, uint32_t N,
                                              uint32_t NS, double rA, double rB) {
    using T = typename PR::T;
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= N) return;
    const SiteGeom g = site_xyz(site, nx, ny);
    const uint32_t e = elem_at(g, 0, 0, 0, nx, ny, nz, px);
    const double rref[2] = {rA, rB};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t x = site_at(g, VSet<Q>::cx(i), VSet<Q>::cy(i), VSet<Q>::cz(i), nx, ny, nz);
        double ux = 0.0, uy = 0.0, uz = 0.0;
        if (u) {
            ux = u[x];
            uy = u[(size_t)N + x];
            uz = u[2 * (size_t)N + x];
        }
        const double cu = VSet<Q>::cx(i) * ux + VSet<Q>::cy(i) * uy + VSet<Q>::cz(i) * uz;
        const double uu = ux * ux + uy * uy + uz * uz;
        const double poly = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double fe = VSet<Q>::w(i) * rho[(size_t)s * N + x] * poly;
            const double val = PR::shifted ? fe - VSet<Q>::w(i) * rref[s] : fe;
            f[(size_t)(s * Q + i) * NS + e] = T(val);
        }
    }
}

hipError_t launch_init(int Q, int prec, void* f, uint32_t NS, const double* rho, const double* u,
                       int nx, int ny, int nz, int px, const double* rho_ref, hipStream_t s) {
    const uint32_t N = (uint32_t)nx * ny * nz;
    const unsigned nblk = (N + 255u) / 256u;
#define SC_INIT(QQ, PP)                                                                      \
    hipLaunchKernelGGL((k_init<QQ, PP>), dim3(nblk), dim3(256), 0, s,                        \
                       static_cast<typename PP::T*>(f), rho, u, nx, ny, nz, px, N, NS,     \
                       rho_ref[0], rho_ref[1])
    if (Q == 9) {
        if (prec == 0) SC_INIT(9, PF64); else SC_INIT(9, PF32S);
    } else {
        if (prec == 0) SC_INIT(19, PF64); else SC_INIT(19, PF32S);
    }
#undef SC_INIT
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Population export / import of one (s, i) array (f points at that array),
// converting the pulled storage to the state f(x, t) (and shifted values back
// to full ones).
// ---------------------------------------------------------------------------
template <int Q, class PR>
__global__ void __launch_bounds__(256) k_get_plane(const typename PR::T* f, double* out, int i,
                                                   int nx, int ny, int nz, int px, uint32_t N,
                                                   double shift) {
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= N) return;
    const SiteGeom g = site_xyz(site, nx, ny);
    const uint32_t src =
        elem_at(g, -VSet<Q>::cx(i), -VSet<Q>::cy(i), -VSet<Q>::cz(i), nx, ny, nz, px);
    out[site] = (double)f[src] + shift;
}

template <int Q, class PR>
__global__ void __launch_bounds__(256) k_set_plane(typename PR::T* f, const double* in, int i,
                                                   int nx, int ny, int nz, int px, uint32_t N,
                                                   double shift) {
    using T = typename PR::T;
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= N) return;
    const SiteGeom g = site_xyz(site, nx, ny);
    const uint32_t src = site_at(g, VSet<Q>::cx(i), VSet<Q>::cy(i), VSet<Q>::cz(i), nx, ny, nz);
    f[elem_at(g, 0, 0, 0, nx, ny, nz, px)] = T(in[src] - shift);
}

hipError_t launch_get_plane(int Q, int prec, const void* f, uint32_t NS, double* out, int s_,
                            int i, int nx, int ny, int nz, int px, const double* rho_ref,
                            hipStream_t s) {
    const uint32_t N = (uint32_t)nx * ny * nz;
    const unsigned nblk = (N + 255u) / 256u;
    const double wi = Q == 9 ? VSet<9>::w(i) : VSet<19>::w(i);
    const double shift = prec == 0 ? 0.0 : wi * rho_ref[s_];
#define SC_GET(QQ, PP)                                                                        \
    hipLaunchKernelGGL((k_get_plane<QQ, PP>), dim3(nblk), dim3(256), 0, s,                    \
                       static_cast<const typename PP::T*>(f) + (size_t)(s_ * QQ + i) * NS, out,  \
                       i, nx, ny, nz, px, N, shift)
    if (Q == 9) {
        if (prec == 0) SC_GET(9, PF64); else SC_GET(9, PF32S);
    } else {
        if (prec == 0) SC_GET(19, PF64); else SC_GET(19, PF32S);
    }
#undef SC_GET
    return hipGetLastError();
}

hipError_t launch_set_plane(int Q, int prec, void* f, uint32_t NS, const double* in, int s_,
                            int i, int nx, int ny, int nz, int px, const double* rho_ref,
                            hipStream_t s) {
    const uint32_t N = (uint32_t)nx * ny * nz;
    const unsigned nblk = (N + 255u) / 256u;
    const double wi = Q == 9 ? VSet<9>::w(i) : VSet<19>::w(i);
    const double shift = prec == 0 ? 0.0 : wi * rho_ref[s_];
#define SC_SET(QQ, PP)                                                                      \
    hipLaunchKernelGGL((k_set_plane<QQ, PP>), dim3(nblk), dim3(256), 0, s,                  \
                       static_cast<typename PP::T*>(f) + (size_t)(s_ * QQ + i) * NS, in, i,  \
                       nx, ny, nz, px, N, shift)
    if (Q == 9) {
        if (prec == 0) SC_SET(9, PF64); else SC_SET(9, PF32S);
    } else {
        if (prec == 0) SC_SET(19, PF64); else SC_SET(19, PF32S);
    }
#undef SC_SET
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 observables.
//   pass 1: rho_s(x) = sum_i f_is(x, t)      (FP64, shifted: rho_ref + sum h)
//   pass 2: j_s, force F_s = -G rho_s sum_i w_i rho_s'(x + c_i) c_i (+ body),
//           u_phys = (j_A + j_B + F/2) / rho, bulk pressure, probe means,
//           phi >= 0 count, non-finite count; per-block partials: a fixed
//           cross-lane butterfly within each wave, then one LDS step over the
//           block's waves
//   pass 3: one block reduces the partials the same way.
// ---------------------------------------------------------------------------
template <int Q, class PR>
__global__ void __launch_bounds__(256) k_rho64(const typename PR::T* f, double* rho, int nx, int ny,
                                               int nz, int px, uint32_t N, uint32_t NS, double rA,
                                               double rB) {
    const uint32_t site = blockIdx.x * 256u + threadIdx.x;
    if (site >= N) return;
    const SiteGeom g = site_xyz(site, nx, ny);
    const double rref[2] = {rA, rB};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            r += (double)f[(size_t)(s * Q + i) * NS +
                           elem_at(g, -VSet<Q>::cx(i), -VSet<Q>::cy(i), -VSet<Q>::cz(i), nx, ny, nz,
                                   px)];
        rho[(size_t)s * N + site] = PR::shifted ? rref[s] + r : r;
    }
}

__device__ __forceinline__ bool is_max_slot(int k) { return k == T_MAX_U; }

// Reduction of one total over the 64 lanes of a wave: a butterfly over lane
// distances 32, 16, ..., 1 (cross-lane permutes, no LDS traffic, no barrier).
// The order of the operations is fixed, so the result is the same on every
// run; lane 0's value is the one used.
__device__ __forceinline__ double wave_reduce(double v, bool is_max) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double o = __shfl_xor(v, m, 64);
        v = is_max ? fmax(v, o) : v + o;
    }
    return v;
}

// Block reduction of the T_COUNT totals: each wave reduces its lanes, then
// one LDS step combines the waves in wave order.  Thread k < T_COUNT returns
// total k.
template <int NT>
__device__ __forceinline__ double block_reduce(double (&v)[T_COUNT], double (&red)[T_COUNT][NT / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < T_COUNT; ++k) {
        const double r = wave_reduce(v[k], is_max_slot(k));
        if (lane == 0) red[k][wave] = r;
    }
    __syncthreads();
    double out = 0.0;
    if ((int)threadIdx.x < T_COUNT) {
        const int k = threadIdx.x;
        out = red[k][0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) out = is_max_slot(k) ? fmax(out, red[k][w]) : out + red[k][w];
    }
    return out;
}

template <int Q, class PR>
__global__ void __launch_bounds__(OBS_BLOCK) k_observe(ObsArgs a) {
    using T = typename PR::T;
    __shared__ double red[T_COUNT][OBS_BLOCK / 64];
    const uint32_t site = blockIdx.x * (uint32_t)OBS_BLOCK + threadIdx.x;
    double v[T_COUNT];
#pragma unroll
    for (int k = 0; k < T_COUNT; ++k) v[k] = 0.0;
    if (site < a.N) {
        const T* f = static_cast<const T*>(a.f);
        const uint32_t N = a.N;
        const SiteGeom g = site_xyz(site, a.nx, a.ny);
        double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double fv =
                    (double)f[(size_t)(s * Q + i) * a.NS +
                              elem_at(g, -VSet<Q>::cx(i), -VSet<Q>::cy(i), -VSet<Q>::cz(i), a.nx,
                                      a.ny, a.nz, a.px)];
                j[0] += VSet<Q>::cx(i) * fv;
                j[1] += VSet<Q>::cy(i) * fv;
                j[2] += VSet<Q>::cz(i) * fv;
            }
        const double rA = a.rho[site], rB = a.rho[(size_t)N + site];
        double gs[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint32_t nb = site_at(g, VSet<Q>::cx(i), VSet<Q>::cy(i), VSet<Q>::cz(i), a.nx,
                                        a.ny, a.nz);
            const double w = VSet<Q>::w(i);
            const double nA = a.rho[nb], nB = a.rho[(size_t)N + nb];
            gs[0][0] += w * nA * VSet<Q>::cx(i);
            gs[0][1] += w * nA * VSet<Q>::cy(i);
            gs[0][2] += w * nA * VSet<Q>::cz(i);
            gs[1][0] += w * nB * VSet<Q>::cx(i);
            gs[1][1] += w * nB * VSet<Q>::cy(i);
            gs[1][2] += w * nB * VSet<Q>::cz(i);
        }
        const double rho = rA + rB;
        double Ft[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) Ft[c] = -a.G * rA * gs[1][c] - a.G * rB * gs[0][c];
        if (a.body_A != 0.0) Ft[0] += rho * a.body_A * sin(2.0 * M_PI * (double)g.y / (double)a.ny);
        double u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) u[c] = (j[c] + 0.5 * Ft[c]) / rho;
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const double umag = sqrt(uu);
        if (a.u) {
            a.u[site] = u[0];
            a.u[(size_t)N + site] = u[1];
            a.u[2 * (size_t)N + site] = u[2];
        }
        const double cs2 = 1.0 / 3.0;
        const double p = cs2 * rho + cs2 * a.G * rA * rB;
        v[T_MASS_A] = rA;
        v[T_MASS_B] = rB;
        v[T_MOM_X] = j[0];
        v[T_MOM_Y] = j[1];
        v[T_MOM_Z] = j[2];
        v[T_MAX_U] = umag;
        v[T_KE] = uu;
        v[T_N_PHI_POS] = (rA - rB >= 0.0) ? 1.0 : 0.0;
        v[T_N_NONFINITE] = (isfinite(rA) && isfinite(rB) && isfinite(uu)) ? 0.0 : 1.0;
        if (a.has_probe) {
            double dx = g.x - a.probe[0], dy = g.y - a.probe[1], dz = g.z - a.probe[2];
            dx -= a.nx * round(dx / a.nx);
            dy -= a.ny * round(dy / a.ny);
            dz = a.nz > 1 ? dz - a.nz * round(dz / a.nz) : 0.0;
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d <= a.r_in) {
                v[T_P_IN] = p;
                v[T_N_IN] = 1.0;
                v[T_RA_IN] = rA;
            } else if (d > a.r_out) {
                v[T_P_OUT] = p;
                v[T_N_OUT] = 1.0;
                v[T_RA_OUT] = rA;
            }
        }
    }
    const double tot = block_reduce<OBS_BLOCK>(v, red);
    if (threadIdx.x < T_COUNT) a.partial[(size_t)blockIdx.x * T_COUNT + threadIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_finalize(const double* partial, int nparts, double* out) {
    __shared__ double red[T_COUNT][256 / 64];
    double v[T_COUNT];
#pragma unroll
    for (int k = 0; k < T_COUNT; ++k) v[k] = 0.0;
    for (int r = threadIdx.x; r < nparts; r += 256) {
#pragma unroll
        for (int k = 0; k < T_COUNT; ++k) {
            const double o = partial[(size_t)r * T_COUNT + k];
            v[k] = is_max_slot(k) ? fmax(v[k], o) : v[k] + o;
        }
    }
    const double tot = block_reduce<256>(v, red);
    if (threadIdx.x < T_COUNT) out[threadIdx.x] = tot;
}

int observe_blocks(uint32_t N) { return (int)((N + OBS_BLOCK - 1) / OBS_BLOCK); }

hipError_t launch_observe(int Q, int prec, const ObsArgs& a, double* totals, hipStream_t s) {
    const unsigned nblk = (unsigned)observe_blocks(a.N);
    double* rho = const_cast<double*>(a.rho);
#define SC_OBS(QQ, PP)                                                                          \
    do {                                                                                        \
        hipLaunchKernelGGL((k_rho64<QQ, PP>), dim3(nblk), dim3(256), 0, s,                      \
                           static_cast<const typename PP::T*>(a.f), rho, a.nx, a.ny, a.nz, a.px,\
                           a.N, a.NS, a.rho_ref[0], a.rho_ref[1]);                              \
        hipLaunchKernelGGL((k_observe<QQ, PP>), dim3(nblk), dim3(OBS_BLOCK), 0, s, a);          \
    } while (0)
    if (Q == 9) {
        if (prec == 0) SC_OBS(9, PF64); else SC_OBS(9, PF32S);
    } else {
        if (prec == 0) SC_OBS(19, PF64); else SC_OBS(19, PF32S);
    }
#undef SC_OBS
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, a.partial, (int)nblk, totals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy (8-byte elements, nontemporal stores): the achievable
// read+write bandwidth of the step's element size.  One element per thread
// and iteration over a grid of up to 2^18 blocks (about four elements per
// thread for 2 GiB): of the grid sizes and unrollings measured on MI355X this
// form moved the most bytes (6.3 TB/s; four loads in flight per thread over
// 2^16 blocks: 5.5 TB/s).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_copy(uint64_t* __restrict__ dst,
                                              const uint64_t* __restrict__ src, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256u;
    for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride)
        store_nt(dst + i, src[i]);
}

hipError_t launch_copy(void* dst, const void* src, size_t nbytes, hipStream_t s) {
    const size_t n = nbytes / 8;
    size_t blocks = (n + 4 * 256 - 1) / (4 * 256);
    if (blocks > (1u << 18)) blocks = 1u << 18;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint64_t*>(dst),
                       static_cast<const uint64_t*>(src), n);
    return hipGetLastError();
}

}  // namespace sc
