// sc_device.h -- device code of the two-component Shan-Chen BGK step for
// gfx950: velocity sets, precision policies and the fused tile-march step
// shared by the single-lattice, batched and persistent launches.
//
// Method (Scarbolo et al., Sec. 2.1, eq:be, moment definitions, eq. FORCE):
//   rho_s = sum_i f_is,  j_s = sum_i f_is c_i
//   a_s   = -G sum_i w_i rho_s'(x + c_i) c_i       (F_s = rho_s a_s, psi = rho)
//   u'    = (j_A/tau_A + j_B/tau_B) / (rho_A/tau_A + rho_B/tau_B)
//   v_s   = u' + tau_s a_s                          (= u' + tau_s F_s / rho_s)
//   f*_is = f_is + (f^eq_is(rho_s, v_s) - f_is) / tau_s
//   f_is(x + c_i, t + 1) = f*_is(x, t)              (periodic)
//
// Memory layout.  Populations are SoA, one contiguous array per (species,
// velocity): buf[(s*Q + i)*NS + e], e = (z*ny + y)*px + x, with x rows px >= nx
// elements apart (rows padded to 32 elements on large lattices, so that each
// row starts on a cache line) and arrays NS >= px*ny*nz apart.  Two buffers
// ping-pong.  A buffer holds post-collision values f*(x, t-1) at x, so the
// state f(x, t) is read "pulled": f_is(x, t) = buf[s][i][x - c_i].  Every
// store is aligned and coalesced; a pulled load is misaligned by at most one
// element along x.
//
// Fused step.  A block owns a transverse tile (TX x TY sites of the xy plane
// on D3Q19, TX sites of an x row on D2Q9) and marches along the slowest axis
// (z on D3Q19, y on D2Q9) over mb planes.  For plane m+1 it pulls the
// populations of its own sites into registers and of a one-site ring around
// the tile, reduces them to densities and keeps the densities of planes m-1,
// m, m+1 (plus one spare) in a 4-slot LDS ring.  Plane m is then collided
// from registers with the force gathered from LDS and stored.  HBM sees each
// population read once and written once per step, plus the ring and the two
// extra planes at chunk ends (served mostly by L2 / MALL).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sc {

// ---------------------------------------------------------------------------
// Velocity sets (export order of the C ABI).
// ---------------------------------------------------------------------------
template <int Q>
struct VSet;

template <>
struct VSet<9> {
    static constexpr int D = 2;
    __host__ __device__ static constexpr int cx(int i) {
        constexpr int a[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        return a[i];
    }
    __host__ __device__ static constexpr int cy(int i) {
        constexpr int a[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return a[i];
    }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};

template <>
struct VSet<19> {
    static constexpr int D = 3;
    __host__ __device__ static constexpr int cx(int i) {
        constexpr int a[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0};
        return a[i];
    }
    __host__ __device__ static constexpr int cy(int i) {
        constexpr int a[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 1, -1};
        return a[i];
    }
    __host__ __device__ static constexpr int cz(int i) {
        constexpr int a[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, -1, 1};
        return a[i];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};

// Index of the velocity opposite to c_i.
template <int Q>
__host__ __device__ constexpr int opposite(int i) {
    for (int k = 0; k < Q; ++k)
        if (VSet<Q>::cx(k) == -VSet<Q>::cx(i) && VSet<Q>::cy(k) == -VSet<Q>::cy(i) &&
            VSet<Q>::cz(k) == -VSet<Q>::cz(i))
            return k;
    return i;
}

// Plane geometry: the march axis is the slowest lattice axis.  A velocity
// moves (dx, dy) inside the plane and dm across planes.
template <int Q>
struct Geo {
    static constexpr bool is3d = (Q == 19);
    static constexpr int HY = is3d ? 1 : 0;  // ring rows above/below the tile
    __host__ __device__ static constexpr int dx(int i) { return VSet<Q>::cx(i); }
    __host__ __device__ static constexpr int dy(int i) { return is3d ? VSet<Q>::cy(i) : 0; }
    __host__ __device__ static constexpr int dm(int i) {
        return is3d ? VSet<Q>::cz(i) : VSet<Q>::cy(i);
    }
};

// ---------------------------------------------------------------------------
// Precision policies.  T: stored type; A: arithmetic type of the collision.
// Shifted storage holds h = f - w_i rho_ref; the density then splits into
// rho_ref + delta with delta = sum_i h (exact cancellation of the large part).
// ---------------------------------------------------------------------------
struct PF64 {
    using T = double;
    using A = double;
    static constexpr bool shifted = false;
    static constexpr bool guo = false;   // force through the velocity shift
    static constexpr bool trt = false;   // one relaxation time (BGK)
    static constexpr int code = 0;
};
struct PF32S {
    using T = float;
    using A = float;
    static constexpr bool shifted = true;
    static constexpr bool guo = false;
    static constexpr bool trt = false;
    static constexpr int code = 1;
};
// The same storage with the Guo discrete forcing (G) and / or two relaxation
// times (T).  The step kernels are instantiated per policy, so no scheme pays
// for another's registers.
struct PF64G : PF64 {
    static constexpr bool guo = true;
};
struct PF32SG : PF32S {
    static constexpr bool guo = true;
};
struct PF64T : PF64 {
    static constexpr bool trt = true;
};
struct PF32ST : PF32S {
    static constexpr bool trt = true;
};
struct PF64GT : PF64G {
    static constexpr bool trt = true;
};
struct PF32SGT : PF32SG {
    static constexpr bool trt = true;
};

// Everything a step of one lattice needs; passed by value into kernels or
// read from a descriptor table by batched launches.
struct StepParams {
    const void* src;
    void* dst;
    int NX, NY, NM;     // transverse extents and march extent
    int PX;             // elements from one x row of a population array to the next (>= NX)
    uint32_t P;         // elements from one plane to the next, PX * NY
    uint32_t N;         // sites
    uint32_t NS;        // elements from one population array to the next (>= N)
    int ntx, nty;       // tiles across the plane
    int nchunks, mb;    // march chunks of mb planes
    int ny_lat;         // lattice y extent (Kolmogorov forcing period)
    double tau[2], omega[2];
    double tau_m[2], omega_m[2];  // odd-part relaxation (= tau, omega for one relaxation time)
    double G;
    double rho_ref[2];
    double body_A;
    int forcing;        // 0: velocity shift (Sec. 2.1), 1: Guo (selects the kernel policy)
};

// Broadcast of block-uniform values into scalar registers.  Batched launches
// read their StepParams from a descriptor table through a per-block index;
// these make the compiler treat the fields as the uniform values they are
// (scalar bases for buffer resources instead of per-lane waterfalls).
__device__ __forceinline__ uint32_t uni32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni32((uint32_t)(x >> 32)) << 32) | uni32((uint32_t)x);
}
__device__ __forceinline__ double unid(double x) {
    return __builtin_bit_cast(double, uni64(__builtin_bit_cast(uint64_t, x)));
}
template <typename P>
__device__ __forceinline__ P* unip(P* x) {
    return reinterpret_cast<P*>(uni64(reinterpret_cast<uint64_t>(x)));
}

__device__ __forceinline__ int wrapi(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ void store_nt(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// A scalar the optimiser may neither hoist nor fold: the per-(s, i) array
// bases derived from it are recomputed where used (a few scalar ops) instead
// of being hoisted out of the plane loop, where 38 of them would overflow the
// SGPR file into VGPRs.
__device__ __forceinline__ uint32_t opaque_sgpr(uint32_t x) {
    asm volatile("; sc opaque %0" : "+s"(x));
    return x;
}

// Raw buffer access.  A resource covers one (species, velocity) array
// (< 4 GiB since N * sizeof(T) < 2^32); soff is a uniform byte offset (the
// plane), voff the lane's byte offset.  Accesses beyond the array read 0 and
// drop stores instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit data format

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kBufWord3);
}

// AUX is the cache policy: 0 = default, 2 = nontemporal (streamed through L2
// at low retention, for data no other block reads again).
template <typename T, int AUX = 0>
__device__ __forceinline__ T buf_load(rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}

// nontemporal store (aux bit 1: streaming, do not keep in L2)
template <typename T>
__device__ __forceinline__ void buf_store_nt(T v, rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ void buf_store_nt<double>(double v, rsrc_t r, uint32_t voff,
                                                     uint32_t soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 2);
}
template <>
__device__ __forceinline__ void buf_store_nt<float>(float v, rsrc_t r, uint32_t voff,
                                                    uint32_t soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), r, voff, soff, 2);
}

// Maps a launch-order block id to a work id so that the blocks the hardware
// places on one XCD (ids congruent mod 8) get a contiguous range of tiles:
// neighbouring tiles then share that XCD's L2 for their ring loads.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    if ((nblk & 7) != 0) return bid;
    return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

__device__ __forceinline__ StepParams uniform_params(const StepParams& q) {
    StepParams p;
    p.src = unip(q.src);
    p.dst = unip(q.dst);
    p.NX = (int)uni32((uint32_t)q.NX);
    p.NY = (int)uni32((uint32_t)q.NY);
    p.NM = (int)uni32((uint32_t)q.NM);
    p.PX = (int)uni32((uint32_t)q.PX);
    p.P = uni32(q.P);
    p.N = uni32(q.N);
    p.NS = uni32(q.NS);
    p.ntx = (int)uni32((uint32_t)q.ntx);
    p.nty = (int)uni32((uint32_t)q.nty);
    p.nchunks = (int)uni32((uint32_t)q.nchunks);
    p.mb = (int)uni32((uint32_t)q.mb);
    p.ny_lat = (int)uni32((uint32_t)q.ny_lat);
    for (int s = 0; s < 2; ++s) {
        p.tau[s] = unid(q.tau[s]);
        p.omega[s] = unid(q.omega[s]);
        p.tau_m[s] = unid(q.tau_m[s]);
        p.omega_m[s] = unid(q.omega_m[s]);
        p.rho_ref[s] = unid(q.rho_ref[s]);
    }
    p.G = unid(q.G);
    p.body_A = unid(q.body_A);
    p.forcing = (int)uni32((uint32_t)q.forcing);
    return p;
}

// Kolmogorov body acceleration A sin(2 pi y / L_y) of Sec. 4.2 at lattice row y.
__device__ __forceinline__ double kolmogorov(const StepParams& p, int y) {
    return p.body_A * sin(2.0 * M_PI * (double)y / (double)p.ny_lat);
}

// Floating-point contraction.  The library is compiled without implicit
// contraction; the fused multiply-adds below are written out, so every launch
// form performs the same IEEE operations in the same order and a lattice
// evolves bitwise the same whichever kernel variant, tile shape or batch
// advances it.
__device__ __forceinline__ double fmaa(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaa(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Force gather of both species, g[s] = sum_{i>0} w_i rho_s(x + c_i) c_i (the
// sum of eq. FORCE without the -G psi_s' factor); rho(s, i) returns the
// density of species s at the neighbour x + c_i.
template <int Q, class A, class Rho>
__device__ __forceinline__ void gather(Rho&& rho, A (&g)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        A gx = A(0), gy = A(0), gz = A(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const A r = rho(s, i);
            const A w = A(VSet<Q>::w(i));
            if (VSet<Q>::cx(i)) gx = fmaa(VSet<Q>::cx(i) > 0 ? w : -w, r, gx);
            if (VSet<Q>::cy(i)) gy = fmaa(VSet<Q>::cy(i) > 0 ? w : -w, r, gy);
            if (VSet<Q>::cz(i)) gz = fmaa(VSet<Q>::cz(i) > 0 ? w : -w, r, gz);
        }
        g[s][0] = gx;
        g[s][1] = gy;
        g[s][2] = gz;
    }
}

// Relaxation and store of species s towards its equilibrium at velocity v.
//   om, omm : 1/tau_s of the even and of the odd part of the deviation from
//             equilibrium (equal for one relaxation time)
//   F       : the species' force, for the Guo source (u = v then)
// One relaxation time: f*_i = f_i + om (feq_i - f_i) [+ Guo source].  Two
// (PR::trt): the same plus (om - omm) / 2 [(f_i - f_ib) - (feq_i - feq_ib)]
// with ib the opposite velocity, which relaxes the odd part with omm; the
// pairs (i, ib) are processed together.  The Guo source's even part
// w_i (9 cu cF - 3 u.F) takes (1 - om/2), its odd part w_i 3 cF (1 - omm/2).
template <int Q, class PR>
__device__ __forceinline__ void relax_store(const typename PR::T (&fs)[Q], int s,
                                            const typename PR::A (&v)[3],
                                            const typename PR::A (&F)[3], typename PR::A rho,
                                            typename PR::A rfull, typename PR::A om,
                                            typename PR::A omm, char* __restrict__ dst,
                                            uint32_t pbytes, uint32_t voff, uint32_t soff) {
    using T = typename PR::T;
    using A = typename PR::A;
    const A vv = fmaa(v[0], v[0], fmaa(v[1], v[1], v[2] * v[2]));
    const A base = fmaa(A(-1.5), vv, A(1));
    // Guo source S_i = w_i [cF (c9 cu + c3) - uF3] with the prefactors folded
    // into c9, c3 and uF3 (two relaxation times) or into the force (one)
    A Fp[3] = {A(0), A(0), A(0)}, uF3 = A(0), c9 = A(9), c3 = A(3);
    if constexpr (PR::guo) {
        const A pe = fmaa(A(-0.5), om, A(1));
        if constexpr (PR::trt) {
#pragma unroll
            for (int a = 0; a < 3; ++a) Fp[a] = F[a];
            c9 = A(9) * pe;
            c3 = A(3) * fmaa(A(-0.5), omm, A(1));
            uF3 = (A(3) * pe) * fmaa(v[0], Fp[0], fmaa(v[1], Fp[1], v[2] * Fp[2]));
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) Fp[a] = pe * F[a];
            uF3 = A(3) * fmaa(v[0], Fp[0], fmaa(v[1], Fp[1], v[2] * Fp[2]));
        }
    }
    // one-relaxation-time update of population i; its equilibrium into feq
    auto post = [&](int i, A& feq) -> A {
        A cu = A(0);
        if (VSet<Q>::cx(i)) cu += VSet<Q>::cx(i) > 0 ? v[0] : -v[0];
        if (VSet<Q>::cy(i)) cu += VSet<Q>::cy(i) > 0 ? v[1] : -v[1];
        if (VSet<Q>::cz(i)) cu += VSet<Q>::cz(i) > 0 ? v[2] : -v[2];
        const A wi = A(VSet<Q>::w(i));
        if (PR::shifted) {
            // h^eq = f^eq - w rho_ref = w [delta + rho (3cu + 4.5cu^2 - 1.5vv)]
            const A poly = fmaa(A(4.5) * cu, cu, fmaa(A(3), cu, A(-1.5) * vv));
            feq = wi * fmaa(rfull, poly, rho);
        } else {
            feq = wi * rfull * fmaa(A(4.5) * cu, cu, fmaa(A(3), cu, base));
        }
        const A fv = A(fs[i]);
        A fo = fmaa(om, feq - fv, fv);
        if constexpr (PR::guo) {
            A cF = A(0);
            if (VSet<Q>::cx(i)) cF += VSet<Q>::cx(i) > 0 ? Fp[0] : -Fp[0];
            if (VSet<Q>::cy(i)) cF += VSet<Q>::cy(i) > 0 ? Fp[1] : -Fp[1];
            if (VSet<Q>::cz(i)) cF += VSet<Q>::cz(i) > 0 ? Fp[2] : -Fp[2];
            // (c_i - u).F / c_S^2 + (c_i.u)(c_i.F) / c_S^4 with c_S^2 = 1/3
            const A t = fmaa(cF, fmaa(c9, cu, c3), -uF3);
            fo = fmaa(wi, t, fo);
        }
        return fo;
    };
    auto store = [&](int i, A fo) {
        buf_store_nt<T>(T(fo), make_rsrc(dst + (size_t)(s * Q + i) * pbytes, pbytes), voff, soff);
    };
    if constexpr (!PR::trt) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            A feq;
            store(i, post(i, feq));
        }
    } else {
        const A hd = A(0.5) * (om - omm);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ib = opposite<Q>(i);
            if (ib < i) continue;
            A ei;
            const A oi = post(i, ei);
            if (ib == i) {
                store(i, oi);
                continue;
            }
            A eb;
            const A ob = post(ib, eb);
            const A B = (A(fs[i]) - A(fs[ib])) - (ei - eb);
            store(i, fmaa(hd, B, oi));
            store(ib, fmaa(-hd, B, ob));
        }
    }
}

// Collision of one site and store of its 2Q post-collision populations.
//   f      : the site's pulled populations f_is(x, t) (shifted h_is in FP32 mode)
//   g[s]   : sum_i w_i rho_s(x + c_i) c_i, the gather of species s
//   body   : external acceleration along x (0 without forcing)
// The force on species s is F_s = rho_s a_s with a_s = -G g[s'] + body x.
// tau-_s below is the odd-part relaxation time (tau_s for one relaxation time).
// Velocity shift (the paper's scheme): the equilibrium of s is taken at
// v_s = u' + tau-_s a_s, u' = sum_s j_s/tau-_s / sum_s rho_s/tau-_s.
// Guo forcing (PR::guo): both species' equilibria at the common
// u = sum_s (j_s + F_s/2)/tau-_s / sum_s rho_s/tau-_s, plus the source
// S_is = (1 - 1/(2 tau_s)) w_i [3 (c_i - u).F_s + 9 (c_i.u)(c_i.F_s)].
// Stores f*_is at byte offset soff + voff of the (s, i) arrays of dst.  Every
// launch form (fused, two-pass, batched, persistent) calls this function, so
// the per-site arithmetic is identical across them.
template <int Q, class PR>
__device__ __forceinline__ void collide_store(const typename PR::T (&f)[2][Q],
                                              const typename PR::A (&g)[2][3],
                                              const StepParams& p, double body,
                                              char* __restrict__ dst, uint32_t pbytes,
                                              uint32_t voff, uint32_t soff) {
    using A = typename PR::A;
    pbytes = opaque_sgpr(pbytes);
    const A om[2] = {A(p.omega[0]), A(p.omega[1])};
    // the odd relaxation times weight the momenta and scale the force shift
    const A omm[2] = {A(p.omega_m[0]), A(p.omega_m[1])};
    const A taum[2] = {A(p.tau_m[0]), A(p.tau_m[1])};
    const A G = A(p.G);
    A rho[2], rfull[2], j[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        A r = A(0), jx = A(0), jy = A(0), jz = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const A fv = A(f[s][i]);
            r += fv;
            if (VSet<Q>::cx(i)) jx += VSet<Q>::cx(i) > 0 ? fv : -fv;
            if (VSet<Q>::cy(i)) jy += VSet<Q>::cy(i) > 0 ? fv : -fv;
            if (VSet<Q>::cz(i)) jz += VSet<Q>::cz(i) > 0 ? fv : -fv;
        }
        rho[s] = r;
        rfull[s] = PR::shifted ? A(p.rho_ref[s]) + r : r;
        j[s][0] = jx;
        j[s][1] = jy;
        j[s][2] = jz;
    }
    // accelerations a_s = -G g[s'] + body (F_s = rho_s a_s)
    const A bx = A(body);
    A acc[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = -G * g[1 - s][a];
        acc[s][0] += bx;
    }
    const A den = fmaa(rfull[0], omm[0], rfull[1] * omm[1]);
    if constexpr (PR::guo) {
        // Guo: common velocity of the momenta corrected by half the force
        A u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const A mA = fmaa(A(0.5) * rfull[0], acc[0][a], j[0][a]);
            const A mB = fmaa(A(0.5) * rfull[1], acc[1][a], j[1][a]);
            u[a] = fmaa(mA, omm[0], mB * omm[1]) / den;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            A F[3], us[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                F[a] = rfull[s] * acc[s][a];
                // an opaque copy per species: keeps the compiler from sharing the
                // c_i.u terms of the two species, whose values would stay live
                // across the first species' relaxation and overflow the registers
                us[a] = u[a];
                asm volatile("" : "+v"(us[a]));
            }
            relax_store<Q, PR>(f[s], s, us, F, rho[s], rfull[s], om[s], omm[s], dst, pbytes, voff,
                               soff);
        }
    } else {
        // velocity shift: common velocity u', then v_s = u' + tau_s a_s
        A u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = fmaa(j[0][a], omm[0], j[1][a] * omm[1]) / den;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            A v[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a] = fmaa(taum[s], acc[s][a], u[a]);
            relax_store<Q, PR>(f[s], s, v, v, rho[s], rfull[s], om[s], omm[s], dst, pbytes, voff,
                               soff);
        }
    }
}

template <int Q, class PR, int TX, int TY>
struct TileStep {
    using T = typename PR::T;
    using A = typename PR::A;
    static constexpr int HY = Geo<Q>::HY;
    static constexpr int FW = TX + 2;
    static constexpr int FH = TY + 2 * HY;
    static constexpr int NT = TX * TY;
    static constexpr int R = HY ? 2 * FW + 2 * TY : 2;  // ring sites
    static constexpr int SLOT = 2 * FH * FW;             // LDS elements per plane
    static constexpr int LDS_ELEMS = 4 * SLOT;
    static_assert(Q == 19 || TY == 1, "D2Q9 tiles are one row");
    static_assert(R <= NT, "ring must fit in one pass of the block");

    __device__ static __forceinline__ int lidx(int slot, int s, int fy, int fx) {
        return ((slot * 2 + s) * FH + fy) * FW + fx;
    }

    // Sum of the Q pulled populations of one species at an in-plane byte
    // offset set (one ring task).
    __device__ static __forceinline__ A pull_species(const char* __restrict__ src,
                                                     uint32_t plane_bytes, int s,
                                                     const uint32_t (&pb)[3],
                                                     const uint32_t (&off)[2 * HY + 1][3]) {
        plane_bytes = opaque_sgpr(plane_bytes);
        T v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const rsrc_t r = make_rsrc(src + (size_t)(s * Q + i) * plane_bytes, plane_bytes);
            v[i] = buf_load<T>(r, off[HY - Geo<Q>::dy(i)][1 - Geo<Q>::dx(i)],
                               pb[1 - Geo<Q>::dm(i)]);
        }
        __builtin_amdgcn_sched_group_barrier(0x020, Q, 0);  // Q VMEM reads first
        A acc = A(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += A(v[i]);
        return acc;
    }

    // Pull the 2Q populations of one site of plane m into v and return the
    // two species' density sums (delta densities when shifted).  pb holds the
    // byte offsets of planes m-1, m, m+1 (uniform across the block) and off
    // the lane's nine in-plane byte offsets (N * sizeof(T) < 2^32), so every
    // load is a scalar base plus one precomputed 32-bit lane offset.
    template <int AUX = 0>
    __device__ static __forceinline__ void pull(const char* __restrict__ src, uint32_t plane_bytes,
                                                const uint32_t (&pb)[3],
                                                const uint32_t (&off)[2 * HY + 1][3],
                                                T (&v)[2][Q], A& d0, A& d1) {
        plane_bytes = opaque_sgpr(plane_bytes);
        // all 2Q loads are issued before any is consumed: the sums below must
        // not let the scheduler serialise them through one register
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const rsrc_t r = make_rsrc(src + (size_t)(s * Q + i) * plane_bytes, plane_bytes);
                v[s][i] = buf_load<T, AUX>(r, off[HY - Geo<Q>::dy(i)][1 - Geo<Q>::dx(i)],
                                           pb[1 - Geo<Q>::dm(i)]);
            }
        __builtin_amdgcn_sched_group_barrier(0x020, 2 * Q, 0);  // 2Q VMEM reads first
        A acc[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            acc[s] = A(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) acc[s] += A(v[s][i]);
        }
        d0 = acc[0];
        d1 = acc[1];
    }

    // One tile column: march planes [m0, m1) of tile (tile_x, tile_y).
    __device__ static __forceinline__ void run(const StepParams& p_in, int tile_x_in, int tile_y_in, int chunk_in,
                               A* __restrict__ lds) {
        const StepParams p = uniform_params(p_in);
        const int tile_x = (int)uni32((uint32_t)tile_x_in);
        const int tile_y = (int)uni32((uint32_t)tile_y_in);
        const int chunk = (int)uni32((uint32_t)chunk_in);
        const char* __restrict__ src = static_cast<const char*>(p.src);
        char* __restrict__ dst = static_cast<char*>(p.dst);
        const uint32_t pbytes = p.NS * (uint32_t)sizeof(T);  // (s, i) array stride in bytes
        const int tid = threadIdx.x;
        const int tx = tid % TX, ty = tid / TX;
        const int X0 = tile_x * TX, Y0 = tile_y * TY;
        const int m0 = chunk * p.mb;
        const int m1 = min(m0 + p.mb, p.NM);
        const int NX = p.NX, NY = p.NY, NM = p.NM, PX = p.PX;
        const uint32_t P = p.P;

        // interior site: frame position (tx, ty) -> periodic lattice position
        const int gx = wrapi(X0 + tx, NX);
        const int gy = HY ? wrapi(Y0 + ty, NY) : 0;
        const bool valid = (X0 + tx < NX) && (!HY || Y0 + ty < NY);
        uint32_t off[2 * HY + 1][3];
#pragma unroll
        for (int a = 0; a < 2 * HY + 1; ++a) {
            const int yy = HY ? wrapi(gy + a - HY, NY) : 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                off[a][b] = (uint32_t)(yy * PX + wrapi(gx + b - 1, NX)) * (uint32_t)sizeof(T);
        }
        // ring site handled by this thread (tid < R)
        const bool ring = tid < R;
        int rlx = 0, rly = 0;
        if (HY) {
            if (tid < FW) {
                rlx = tid - 1;
                rly = -1;
            } else if (tid < 2 * FW) {
                rlx = tid - FW - 1;
                rly = TY;
            } else if (tid < 2 * FW + TY) {
                rlx = -1;
                rly = tid - 2 * FW;
            } else {
                rlx = TX;
                rly = tid - 2 * FW - TY;
            }
        } else {
            rlx = (tid == 0) ? -1 : TX;
        }
        uint32_t roff[2 * HY + 1][3];
        {
            const int rgx = wrapi(X0 + rlx, NX);
            const int rgy = HY ? wrapi(Y0 + rly, NY) : 0;
#pragma unroll
            for (int a = 0; a < 2 * HY + 1; ++a) {
                const int yy = HY ? wrapi(rgy + a - HY, NY) : 0;
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    roff[a][b] = (uint32_t)(yy * PX + wrapi(rgx + b - 1, NX)) * (uint32_t)sizeof(T);
            }
        }
        const int own_fx = tx + 1, own_fy = ty + HY;
        const uint32_t own_voff = (uint32_t)(gy * PX + gx) * (uint32_t)sizeof(T);
        const int ring_fx = rlx + 1, ring_fy = rly + HY;

        T cur[2][Q], nxt[2][Q];
        A dA, dB;
        uint32_t pb[3];

        auto plane_bases = [&](int m) {
            const int mm = wrapi(m, NM);
            const uint32_t PB = P * (uint32_t)sizeof(T);
            pb[0] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == 0 ? NM - 1 : mm - 1) * PB);
            pb[1] = __builtin_amdgcn_readfirstlane((uint32_t)mm * PB);
            pb[2] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == NM - 1 ? 0 : mm + 1) * PB);
        };
        // densities of the ring and of the interior of plane m into LDS slot
        auto fill_plane = [&](int m, int slot) {
            plane_bases(m);
            if constexpr (HY != 0) {
                // D3Q19: the interior first; by the time the ring is pulled,
                // the neighbouring tiles' interior loads (the same data) have
                // brought much of it into L2.  The ring one species at a
                // time: at most Q more live values next to the two register
                // planes.  (256^3 FP64 2.24 -> 2.18 ms.)
                pull<0>(src, pbytes, pb, off, nxt, dA, dB);
                lds[lidx(slot, 0, own_fy, own_fx)] = dA;
                lds[lidx(slot, 1, own_fy, own_fx)] = dB;
                __builtin_amdgcn_sched_barrier(0);
                if (ring) {
#pragma unroll
                    for (int s = 0; s < 2; ++s)
                        lds[lidx(slot, s, ring_fy, ring_fx)] =
                            pull_species(src, pbytes, s, pb, roff);
                }
            } else {
                // D2Q9 (a two-site ring): the ring first, then the interior
                // (2 % faster than the other order on a batch of 64 lattices)
                if (ring) {
                    T dummy[2][Q];
                    A rA, rB;
                    pull(src, pbytes, pb, roff, dummy, rA, rB);
                    lds[lidx(slot, 0, ring_fy, ring_fx)] = rA;
                    lds[lidx(slot, 1, ring_fy, ring_fx)] = rB;
                }
                // keep the ring's loads from overlapping the plane kept in
                // registers: bounds the live registers to two planes
                __builtin_amdgcn_sched_barrier(0);
                pull<0>(src, pbytes, pb, off, nxt, dA, dB);
                lds[lidx(slot, 0, own_fy, own_fx)] = dA;
                lds[lidx(slot, 1, own_fy, own_fx)] = dB;
            }
        };

        // prologue: planes m0-1 (densities only) and m0 (kept in registers)
        fill_plane(m0 - 1, 0);
        fill_plane(m0, 1);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];

        for (int m = m0; m < m1; ++m) {
            const int k = m - m0;
            fill_plane(m + 1, (k + 2) & 3);
            __syncthreads();
            if (valid) {
                // force gather from the LDS density planes m-1, m, m+1
                A g[2][3];
                gather<Q>([&](int s, int i) {
                    const int slot = (k + 1 + Geo<Q>::dm(i)) & 3;
                    return lds[lidx(slot, s, own_fy + Geo<Q>::dy(i), own_fx + Geo<Q>::dx(i))];
                }, g);
                const double body = p.body_A != 0.0 ? kolmogorov(p, HY ? gy : m) : 0.0;
                collide_store<Q, PR>(cur, g, p, body, dst, pbytes, own_voff,
                                     __builtin_amdgcn_readfirstlane((uint32_t)m * P *
                                                                    (uint32_t)sizeof(T)));
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
        }
    }
};

// ---------------------------------------------------------------------------
// Pipelined march.  Same tile / march / LDS-ring structure as TileStep, but
// three planes of populations live in registers: while plane m is collided,
// the loads of plane m+2 are already in flight, so each wave overlaps its own
// memory latency with its collision instead of waiting at the barrier.  The
// ring densities are split into (site, species) tasks of Q loads spread over
// all threads of the block.
// ---------------------------------------------------------------------------
template <int Q, class PR, int TX, int TY>
struct TileStepPipe {
    using T = typename PR::T;
    using A = typename PR::A;
    using Base = TileStep<Q, PR, TX, TY>;
    static constexpr int HY = Geo<Q>::HY;
    static constexpr int FW = TX + 2;
    static constexpr int FH = TY + 2 * HY;
    static constexpr int NT = TX * TY;
    static constexpr int R = Base::R;
    // Ring (site, species) tasks are dealt out per wave so that a wave's
    // species is uniform and its buffer resources stay scalar (a per-lane
    // species would turn every ring load into a waterfall loop): wave task
    // wt covers species wt & 1 of ring sites (wt >> 1) * 64 + lane.
    static constexpr int NW = NT / 64;                      // waves per block
    static constexpr int RW = (R + 63) / 64;                // waves per species
    static constexpr int RPT = (2 * RW + NW - 1) / NW;      // ring tasks per thread
    static_assert(NT % 64 == 0, "tiles hold whole waves");
    static constexpr int LDS_ELEMS = Base::LDS_ELEMS;

    __device__ static __forceinline__ int lidx(int slot, int s, int fy, int fx) {
        return Base::lidx(slot, s, fy, fx);
    }

    // ring site k -> frame position
    __device__ static __forceinline__ void ring_pos(int k, int& lx, int& ly) {
        if (HY) {
            if (k < FW) {
                lx = k - 1;
                ly = -1;
            } else if (k < 2 * FW) {
                lx = k - FW - 1;
                ly = TY;
            } else if (k < 2 * FW + TY) {
                lx = -1;
                ly = k - 2 * FW;
            } else {
                lx = TX;
                ly = k - 2 * FW - TY;
            }
        } else {
            lx = k == 0 ? -1 : TX;
            ly = 0;
        }
    }

    __device__ static __forceinline__ A pull_species(const char* __restrict__ src,
                                                     uint32_t plane_bytes, int s,
                                                     const uint32_t (&pb)[3],
                                                     const uint32_t (&off)[2 * HY + 1][3]) {
        return Base::pull_species(src, plane_bytes, s, pb, off);
    }

    __device__ static __forceinline__ void run(const StepParams& p_in, int tile_x_in,
                                               int tile_y_in, int chunk_in, A* __restrict__ lds) {
        const StepParams p = uniform_params(p_in);
        const int tile_x = (int)uni32((uint32_t)tile_x_in);
        const int tile_y = (int)uni32((uint32_t)tile_y_in);
        const int chunk = (int)uni32((uint32_t)chunk_in);
        const char* __restrict__ src = static_cast<const char*>(p.src);
        char* __restrict__ dst = static_cast<char*>(p.dst);
        const uint32_t pbytes = p.NS * (uint32_t)sizeof(T);
        const int tid = threadIdx.x;
        const int tx = tid % TX, ty = tid / TX;
        const int X0 = tile_x * TX, Y0 = tile_y * TY;
        const int m0 = chunk * p.mb;
        const int m1 = min(m0 + p.mb, p.NM);
        const int NX = p.NX, NY = p.NY, NM = p.NM, PX = p.PX;
        const uint32_t P = p.P;

        const int gx = wrapi(X0 + tx, NX);
        const int gy = HY ? wrapi(Y0 + ty, NY) : 0;
        const bool valid = (X0 + tx < NX) && (!HY || Y0 + ty < NY);
        uint32_t off[2 * HY + 1][3];
#pragma unroll
        for (int a = 0; a < 2 * HY + 1; ++a) {
            const int yy = HY ? wrapi(gy + a - HY, NY) : 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                off[a][b] = (uint32_t)(yy * PX + wrapi(gx + b - 1, NX)) * (uint32_t)sizeof(T);
        }
        // ring tasks of this thread: wave task (tid / 64) + k * NW
        uint32_t roff[RPT][2 * HY + 1][3];
        int rfx[RPT], rfy[RPT], rsp[RPT];
        bool rok[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int wt = (int)uni32((uint32_t)(tid >> 6)) + k * NW;
            const int site0 = (wt >> 1) * 64 + (tid & 63);
            rok[k] = wt < 2 * RW && site0 < R;
            const int site = rok[k] ? site0 : 0;
            rsp[k] = wt & 1;
            int lx, ly;
            ring_pos(site, lx, ly);
            rfx[k] = lx + 1;
            rfy[k] = ly + HY;
            const int rgx = wrapi(X0 + lx, NX);
            const int rgy = HY ? wrapi(Y0 + ly, NY) : 0;
#pragma unroll
            for (int a = 0; a < 2 * HY + 1; ++a) {
                const int yy = HY ? wrapi(rgy + a - HY, NY) : 0;
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    roff[k][a][b] = (uint32_t)(yy * PX + wrapi(rgx + b - 1, NX)) * (uint32_t)sizeof(T);
            }
        }
        const int own_fx = tx + 1, own_fy = ty + HY;
        const uint32_t own_voff = (uint32_t)(gy * PX + gx) * (uint32_t)sizeof(T);
        auto slot_of = [&](int m) { return (m - m0 + 1) & 3; };
        auto bases = [&](int m, uint32_t (&pb)[3]) {
            const int mm = wrapi(m, NM);
            const uint32_t PB = P * (uint32_t)sizeof(T);
            pb[0] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == 0 ? NM - 1 : mm - 1) * PB);
            pb[1] = __builtin_amdgcn_readfirstlane((uint32_t)mm * PB);
            pb[2] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == NM - 1 ? 0 : mm + 1) * PB);
        };
        auto ring_fill = [&](int m) {
            uint32_t pb[3];
            bases(m, pb);
            const int slot = slot_of(m);
#pragma unroll
            for (int k = 0; k < RPT; ++k)
                if (rok[k])
                    lds[lidx(slot, rsp[k], rfy[k], rfx[k])] =
                        pull_species(src, pbytes, rsp[k], pb, roff[k]);
        };
        auto own_fill = [&](int m, T (&v)[2][Q]) {
            uint32_t pb[3];
            bases(m, pb);
            A dA, dB;
            Base::template pull<0>(src, pbytes, pb, off, v, dA, dB);
            const int slot = slot_of(m);
            lds[lidx(slot, 0, own_fy, own_fx)] = dA;
            lds[lidx(slot, 1, own_fy, own_fx)] = dB;
        };

        T r0[2][Q], r1[2][Q], r2[2][Q];
        // prologue: densities of m0-1, pops (kept) and densities of m0, m0+1
        own_fill(m0 - 1, r2);
        ring_fill(m0 - 1);
        own_fill(m0, r0);
        ring_fill(m0);
        own_fill(m0 + 1, r1);
        ring_fill(m0 + 1);
        __syncthreads();

        for (int m = m0; m < m1; ++m) {
            const bool more = m + 2 <= m1;
            uint32_t pb2[3];
            A d2A = A(0), d2B = A(0);
            A rs[RPT];
            if (more) {
                // issue plane m+2 now; consumed after the collision of plane m
                bases(m + 2, pb2);
                Base::template pull<0>(src, pbytes, pb2, off, r2, d2A, d2B);
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    rs[k] = rok[k] ? pull_species(src, pbytes, rsp[k], pb2, roff[k]) : A(0);
            }
            if (valid) {
                const int km = slot_of(m);
                A g[2][3];
                gather<Q>([&](int s, int i) {
                    const int slot = (km + Geo<Q>::dm(i)) & 3;
                    return lds[lidx(slot, s, own_fy + Geo<Q>::dy(i), own_fx + Geo<Q>::dx(i))];
                }, g);
                const double body = p.body_A != 0.0 ? kolmogorov(p, HY ? gy : m) : 0.0;
                collide_store<Q, PR>(r0, g, p, body, dst, pbytes, own_voff,
                                     __builtin_amdgcn_readfirstlane((uint32_t)m * P *
                                                                    (uint32_t)sizeof(T)));
            }
            if (more) {
                const int s2 = slot_of(m + 2);
                lds[lidx(s2, 0, own_fy, own_fx)] = d2A;
                lds[lidx(s2, 1, own_fy, own_fx)] = d2B;
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    if (rok[k]) lds[lidx(s2, rsp[k], rfy[k], rfx[k])] = rs[k];
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    r0[s][i] = r1[s][i];
                    r1[s][i] = r2[s][i];
                }
        }
    }
};

// ---------------------------------------------------------------------------
// Re-pull march.  Same tile / march / LDS ring as TileStep, but no plane is
// held in registers across iterations: the densities of plane m+1 are summed
// from pulled loads as they arrive, then plane m is pulled again (its reuse
// distance is one plane iteration, a few tens of MB across the GPU, so it is
// served by L2 / the 256 MB Infinity Cache rather than HBM) and collided.
// Holding one plane instead of two halves the registers per thread and
// doubles the waves, and with them the loads in flight per CU.
// ---------------------------------------------------------------------------
template <int Q, class PR, int TX, int TY>
struct TileStepRepull {
    using T = typename PR::T;
    using A = typename PR::A;
    using Base = TileStep<Q, PR, TX, TY>;
    using Pipe = TileStepPipe<Q, PR, TX, TY>;
    static constexpr int HY = Geo<Q>::HY;
    static constexpr int FW = TX + 2;
    static constexpr int FH = TY + 2 * HY;
    static constexpr int NT = TX * TY;
    static constexpr int RPT = Pipe::RPT;
    static constexpr int R = Pipe::R, NW = Pipe::NW, RW = Pipe::RW;
    static constexpr int LDS_ELEMS = Base::LDS_ELEMS;

    // density of one species from Q pulled loads, summed as they arrive
    __device__ static __forceinline__ A dens(const char* __restrict__ src, uint32_t plane_bytes,
                                             int s, const uint32_t (&pb)[3],
                                             const uint32_t (&off)[2 * HY + 1][3]) {
        return Pipe::pull_species(src, plane_bytes, s, pb, off);
    }

    __device__ static __forceinline__ void run(const StepParams& p_in, int tile_x_in,
                                               int tile_y_in, int chunk_in, A* __restrict__ lds) {
        const StepParams p = uniform_params(p_in);
        const int tile_x = (int)uni32((uint32_t)tile_x_in);
        const int tile_y = (int)uni32((uint32_t)tile_y_in);
        const int chunk = (int)uni32((uint32_t)chunk_in);
        const char* __restrict__ src = static_cast<const char*>(p.src);
        char* __restrict__ dst = static_cast<char*>(p.dst);
        const uint32_t pbytes = p.NS * (uint32_t)sizeof(T);
        const int tid = threadIdx.x;
        const int tx = tid % TX, ty = tid / TX;
        const int X0 = tile_x * TX, Y0 = tile_y * TY;
        const int m0 = chunk * p.mb;
        const int m1 = min(m0 + p.mb, p.NM);
        const int NX = p.NX, NY = p.NY, NM = p.NM, PX = p.PX;
        const uint32_t P = p.P;

        const int gx = wrapi(X0 + tx, NX);
        const int gy = HY ? wrapi(Y0 + ty, NY) : 0;
        const bool valid = (X0 + tx < NX) && (!HY || Y0 + ty < NY);
        uint32_t off[2 * HY + 1][3];
#pragma unroll
        for (int a = 0; a < 2 * HY + 1; ++a) {
            const int yy = HY ? wrapi(gy + a - HY, NY) : 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                off[a][b] = (uint32_t)(yy * PX + wrapi(gx + b - 1, NX)) * (uint32_t)sizeof(T);
        }
        uint32_t roff[RPT][2 * HY + 1][3];
        int rfx[RPT], rfy[RPT], rsp[RPT];
        bool rok[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int wt = (int)uni32((uint32_t)(tid >> 6)) + k * NW;
            const int site0 = (wt >> 1) * 64 + (tid & 63);
            rok[k] = wt < 2 * RW && site0 < R;
            const int site = rok[k] ? site0 : 0;
            rsp[k] = wt & 1;
            int lx, ly;
            Pipe::ring_pos(site, lx, ly);
            rfx[k] = lx + 1;
            rfy[k] = ly + HY;
            const int rgx = wrapi(X0 + lx, NX);
            const int rgy = HY ? wrapi(Y0 + ly, NY) : 0;
#pragma unroll
            for (int a = 0; a < 2 * HY + 1; ++a) {
                const int yy = HY ? wrapi(rgy + a - HY, NY) : 0;
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    roff[k][a][b] = (uint32_t)(yy * PX + wrapi(rgx + b - 1, NX)) * (uint32_t)sizeof(T);
            }
        }
        const int own_fx = tx + 1, own_fy = ty + HY;
        const uint32_t own_voff = (uint32_t)(gy * PX + gx) * (uint32_t)sizeof(T);
        auto slot_of = [&](int m) { return (m - m0 + 1) & 3; };
        auto bases = [&](int m, uint32_t (&pb)[3]) {
            const int mm = wrapi(m, NM);
            const uint32_t PB = P * (uint32_t)sizeof(T);
            pb[0] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == 0 ? NM - 1 : mm - 1) * PB);
            pb[1] = __builtin_amdgcn_readfirstlane((uint32_t)mm * PB);
            pb[2] = __builtin_amdgcn_readfirstlane((uint32_t)(mm == NM - 1 ? 0 : mm + 1) * PB);
        };
        // densities of plane m (interior and ring) into its LDS slot
        auto dens_fill = [&](int m) {
            uint32_t pb[3];
            bases(m, pb);
            const int slot = slot_of(m);
#pragma unroll
            for (int k = 0; k < RPT; ++k)
                if (rok[k]) lds[Base::lidx(slot, rsp[k], rfy[k], rfx[k])] = dens(src, pbytes, rsp[k], pb, roff[k]);
            lds[Base::lidx(slot, 0, own_fy, own_fx)] = dens(src, pbytes, 0, pb, off);
            lds[Base::lidx(slot, 1, own_fy, own_fx)] = dens(src, pbytes, 1, pb, off);
        };

        dens_fill(m0 - 1);
        dens_fill(m0);
        T cur[2][Q];
        for (int m = m0; m < m1; ++m) {
            dens_fill(m + 1);
            // plane m again, for the collision (cache-served)
            uint32_t pb[3];
            bases(m, pb);
            A dA, dB;
            Base::template pull<2>(src, pbytes, pb, off, cur, dA, dB);  // last use of plane m
            __syncthreads();
            if (valid) {
                const int km = slot_of(m);
                A g[2][3];
                gather<Q>([&](int s, int i) {
                    const int slot = (km + Geo<Q>::dm(i)) & 3;
                    return lds[Base::lidx(slot, s, own_fy + Geo<Q>::dy(i), own_fx + Geo<Q>::dx(i))];
                }, g);
                const double body = p.body_A != 0.0 ? kolmogorov(p, HY ? gy : m) : 0.0;
                collide_store<Q, PR>(cur, g, p, body, dst, pbytes, own_voff,
                                     __builtin_amdgcn_readfirstlane((uint32_t)m * P *
                                                                    (uint32_t)sizeof(T)));
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Site helpers for the simple (one thread per site) kernels.
// ---------------------------------------------------------------------------
struct SiteGeom {
    int x, y, z;
};

__device__ __forceinline__ SiteGeom site_xyz(uint32_t site, int nx, int ny) {
    SiteGeom g;
    g.x = (int)(site % (uint32_t)nx);
    const uint32_t r = site / (uint32_t)nx;
    g.y = (int)(r % (uint32_t)ny);
    g.z = (int)(r / (uint32_t)ny);
    return g;
}

__device__ __forceinline__ uint32_t site_at(const SiteGeom& g, int dx, int dy, int dz, int nx,
                                            int ny, int nz) {
    const int x = wrapi(g.x + dx, nx), y = wrapi(g.y + dy, ny), z = wrapi(g.z + dz, nz);
    return ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)nx + (uint32_t)x;
}

// The same neighbour's element in a population array whose x rows are px
// elements apart (px >= nx; the columns from nx on are padding).
__device__ __forceinline__ uint32_t elem_at(const SiteGeom& g, int dx, int dy, int dz, int nx,
                                            int ny, int nz, int px) {
    const int x = wrapi(g.x + dx, nx), y = wrapi(g.y + dy, ny), z = wrapi(g.z + dz, nz);
    return ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)px + (uint32_t)x;
}

}  // namespace sc
