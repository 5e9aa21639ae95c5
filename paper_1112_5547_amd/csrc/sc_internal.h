// sc_internal.h -- host-side interface between the runtime / batch engine and
// the kernel translation units of the Shan-Chen library (not exported).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sc_device.h"

namespace sc {

// Number of FP64 totals accumulated by the observables reduction.
enum {
    T_MASS_A, T_MASS_B, T_MOM_X, T_MOM_Y, T_MOM_Z, T_MAX_U, T_KE, T_P_IN, T_N_IN, T_P_OUT,
    T_N_OUT, T_RA_IN, T_RA_OUT, T_N_PHI_POS, T_N_NONFINITE, T_PAD, T_COUNT
};
constexpr int OBS_BLOCK = 256;

struct ObsArgs {
    const void* f;         // current population buffer (pulled read)
    const double* rho;     // FP64 densities [2][N] (written by the density pass)
    double* u;             // u_phys [3][N] or null
    double* partial;       // [nblocks][T_COUNT]
    int nx, ny, nz;
    int px;                // population row pitch (elements from one x row to the next)
    uint32_t N;
    uint32_t NS;           // population array stride (elements)
    double G, body_A;
    double rho_ref[2];
    int has_probe;
    double probe[4];       // cx, cy, cz, R
    double r_in, r_out;    // radius of the inner ball / of the outer boundary
};

// tile tables (shared by runtime and batch engine)
int tile_count(int Q);
bool tile_get(int Q, int k, int* tx, int* ty);
bool tile_supported(int Q, int tx, int ty);

// Step-kernel policy index: storage precision (0 FP64, 1 FP32 shifted), + 2
// for the Guo forcing, + 4 for two relaxation times, in the order
// PF64, PF32S, PF64G, PF32SG, PF64T, PF32ST, PF64GT, PF32SGT.
constexpr int kPolicies = 8;
inline int step_policy(int precision, int forcing, bool trt) {
    return precision + 2 * (forcing != 0) + 4 * (trt ? 1 : 0);
}

// Batched launches: per-lattice descriptor, work item and the sync words of
// the persistent form.
struct BatchDesc {
    StepParams sp[2];  // parity 0 / 1 (source and destination swapped)
    int Q;
    int base_parity;   // buffer holding the state at epoch start
    int steps;         // steps of this epoch
    int pad;
};

struct WorkItem {
    int member, tile_x, tile_y, chunk;
};

// sync words: [0] barrier count (block groups arrived), [1] barrier
// generation, [2] timeout flag; from SYNC_GRP the arrival counters of the
// block groups (kBarrierGroup blocks each, one 64-byte line per counter, so
// that arrivals spread over many addresses instead of queueing on one); from
// SYNC_CTR the per-step work claim counters.  The timeout flag is sticky: the
// per-launch clear leaves it alone, so a give-up stays visible until the
// host has read it.
constexpr int kSyncLine = 16;  // words per 64-byte line
constexpr int kBarrierGroup = 16, kBarrierGroups = 256;
constexpr int kMaxPersistentBlocks = kBarrierGroup * kBarrierGroups;
constexpr int SYNC_COUNT = 0, SYNC_GEN = 1, SYNC_TIMEOUT = 2;
constexpr int SYNC_GRP = kSyncLine;
constexpr int SYNC_CTR = SYNC_GRP + kBarrierGroups * kSyncLine;
constexpr unsigned kSpinLimit = 1u << 26;  // ~seconds of s_sleep polling per barrier

using BatchStepFn = void (*)(const BatchDesc*, const WorkItem*, int, int);
using BatchPersFn = void (*)(const BatchDesc*, const WorkItem*, int, int, unsigned*, unsigned);

// single-lattice step of policy pol (variant 0 fused, 1 two-pass, 2 pipelined,
// 3 re-pull); batch kernels of policy pol for a block shape
hipError_t launch_step(int variant, int Q, int pol, int tx, int ty, const StepParams& p,
                       void* psi, hipStream_t s);
bool batch_kernels(int pol, int nt, int tx19, int ty19, BatchStepFn* sf, BatchPersFn* pf);
// Population buffers hold 2Q arrays of NS >= px ny nz elements (array (s, i)
// at element (s Q + i) NS; site (x, y, z) at element (z ny + y) px + x, with
// x rows px >= nx elements apart).  Host-side fields (rho, u, in, out) hold
// one element per site, (z ny + y) nx + x.
hipError_t launch_init(int Q, int prec, void* f, uint32_t NS, const double* rho, const double* u,
                       int nx, int ny, int nz, int px, const double* rho_ref, hipStream_t s);
hipError_t launch_get_plane(int Q, int prec, const void* f, uint32_t NS, double* out, int s_,
                            int i, int nx, int ny, int nz, int px, const double* rho_ref,
                            hipStream_t s);
hipError_t launch_set_plane(int Q, int prec, void* f, uint32_t NS, const double* in, int s_,
                            int i, int nx, int ny, int nz, int px, const double* rho_ref,
                            hipStream_t s);
hipError_t launch_observe(int Q, int prec, const ObsArgs& a, double* totals, hipStream_t s);
int observe_blocks(uint32_t N);
hipError_t launch_copy(void* dst, const void* src, size_t nbytes, hipStream_t s);

}  // namespace sc
