/*
 * lbm_sc.h -- C ABI of the MI355X (gfx950) two-component Shan-Chen lattice
 * Boltzmann library.
 *
 * The library advances periodic D2Q9 / D3Q19 lattices carrying two species
 * A and B under the multicomponent Shan-Chen BGK equation of Scarbolo et al.,
 * "Unified framework for a side-by-side comparison of different
 * multicomponent algorithms: lattice Boltzmann vs. phase field model",
 * Sec. 2.1 (eq:be, the moment definitions and eq. FORCE):
 *
 *   f_is(x + c_i, t + 1) - f_is(x, t) = -(f_is - f_is^eq(rho_s, u + tau_s F_s / rho_s)) / tau_s
 *   rho_s = sum_i f_is,   u = sum_s (1/tau_s) sum_i f_is c_i / sum_s (1/tau_s) rho_s
 *   F_s(x) = -G rho_s(x) sum_i w_i rho_s'(x + c_i) c_i      (psi = rho, s' != s)
 *
 * with the second-order equilibrium
 *   f_i^eq(rho, v) = w_i rho [1 + 3 c_i.v + 9/2 (c_i.v)^2 - 3/2 v.v]   (c_S^2 = 1/3).
 *
 * Every step runs on the GPU in hand-written HIP kernels; the host only
 * launches them.  No entry point uses a CPU fallback.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Status: every int-returning call returns LBM_OK (0) or a negative
 *   LBM_E* code; lbm_sc_strerror() names it.  A device error is sticky: after
 *   LBM_EDEVICE the handle only accepts lbm_sc_destroy().
 * - Site order: x fastest, then y, then z; N = nx * ny * nz.  Host density
 *   arrays have N doubles.  Velocity fields have 3 * N doubles, component
 *   major (u_x[N], u_y[N], u_z[N]).  Population arrays have 2 * Q * N
 *   doubles ordered [s][i][z][y][x] (species A = 0, B = 1).
 * - Velocity order (export contract):
 *   D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *   D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *          (1,1,0) (-1,-1,0) (1,0,1) (-1,0,-1) (0,1,1) (0,-1,-1)
 *          (1,-1,0) (-1,1,0) (1,0,-1) (-1,0,1) (0,1,-1) (0,-1,1)
 *   Weights: D2Q9 4/9, 1/9 (axis), 1/36 (diagonal); D3Q19 1/3, 1/18, 1/36.
 *   These meet the paper's second- and fourth-order isotropy conditions.
 * - The population state between steps is f(x, t) after streaming and before
 *   collision; lbm_sc_get_populations() returns exactly that.
 * - Ownership: host arrays belong to the caller and are copied during the
 *   call.  Device memory belongs to the handle, or to the caller when an
 *   arena is passed to lbm_sc_create_ex (it must outlive the handle).
 * - Threads: a handle is not thread-safe; distinct handles are independent.
 * - Asynchrony: lbm_sc_step() only enqueues work on the handle's stream.
 *   Calls that return host data synchronise that stream.
 */
#ifndef LBM_SC_H
#define LBM_SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sc lbm_sc;
typedef struct lbm_batch lbm_batch;

enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19 };

/* LBM_FP64: populations stored and collided in double precision.
 * LBM_FP32_SHIFTED: populations stored and collided in single precision as
 * h_is = f_is - w_i rho_ref_s (a per-species FP64 reference density); the
 * moments, observables and reductions are still evaluated in FP64. */
enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 };

/* How the force F_s = psi_s a_s (+ the body force) enters the collision.
 * LBM_FORCING_SHIFT: the paper's scheme (Sec. 2.1, eq:be): the equilibrium
 *   of species s is taken at v_s = u' + tau_s F_s / rho_s, with the common
 *   velocity u' = sum_s j_s / tau_s / sum_s rho_s / tau_s.  Its effective
 *   coupling in the hydrodynamic limit is g^(tau) = tau g / (tau - 1/2).
 * LBM_FORCING_GUO: the discrete forcing of Guo, Zheng and Shi, which the
 *   paper cites as the way to remove that tau-dependence (Sec. 2.3; the paper
 *   gives no formula, this is the standard per-species form):
 *     u     = sum_s (j_s + F_s / 2) / tau_s / sum_s rho_s / tau_s
 *     f*_is = f_is - (f_is - f^eq_is(rho_s, u)) / tau_s + S_is
 *     S_is  = (1 - 1/(2 tau_s)) w_i [ (c_i - u).F_s / c_S^2
 *                                     + (c_i.u)(c_i.F_s) / c_S^4 ]
 *   Each species' mass is conserved and the momentum grows by exactly
 *   sum_s F_s per step; the effective coupling is the bare g. */
enum { LBM_FORCING_SHIFT = 0, LBM_FORCING_GUO = 1 };

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument */
    LBM_ENOMEM = -2,      /* device allocation failed or arena too small */
    LBM_EDEVICE = -3,     /* HIP runtime error (sticky) */
    LBM_ESTATE = -4,      /* call out of order (e.g. step before init) */
    LBM_ENONFINITE = -5,  /* a reduced total is NaN or Inf */
    LBM_EBUDGET = -6,     /* a batch has no room for the lattice */
    LBM_ETIMEOUT = -7,    /* a persistent launch hit its grid-barrier spin limit */
    LBM_ETOOBIG = -8      /* beyond the allocation-free batch run's fixed scratch */
};

/* Lattice parameters.  Validation (LBM_EINVAL otherwise):
 *   lattice in {LBM_D2Q9, LBM_D3Q19}; nx, ny, nz >= 1; nz == 1 for D2Q9;
 *   N = nx*ny*nz <= 2^29 - 2112 (32-bit population offsets, array padding
 *   included);
 *   tau_A, tau_B > 1/2 (positive viscosity c_S^2 (tau - 1/2), Sec. 2.1);
 *   G >= 0 (g_AB > 0 is the repulsive coupling, Sec. 2.1; 0 decouples);
 *   rho_ref_A, rho_ref_B: FP32_SHIFTED reference densities; a value <= 0
 *   means "the volume mean of the densities passed to lbm_sc_init";
 *   body_A: amplitude A of the Kolmogorov body force of Sec. 4.2,
 *   F_x += rho_s A sin(2 pi y / ny) on each species (0 disables it);
 *   forcing: LBM_FORCING_SHIFT (default) or LBM_FORCING_GUO;
 *   tau_minus_A, tau_minus_B: relaxation time of the odd part (under
 *   c_i -> -c_i) of each species' deviation from equilibrium, > 1/2; a value
 *   <= 0 means tau_s (the paper's single-relaxation-time BGK, eq:be).  A
 *   different value is the two-relaxation-time member of the
 *   multiple-relaxation-time family the paper names for decoupling the
 *   diffusive and viscous time scales (Sec. 2.1, closing remark):
 *     f*_is = f_is - (f+_is - feq+_is) / tau_s - (f-_is - feq-_is) / tau-_s,
 *     f+-_i = (f_i +- f_ibar) / 2 (ibar: the velocity opposite to i),
 *   with the momentum weights and the force shift (or Guo's odd source part)
 *   taken with tau-_s.  The viscosity is c_S^2 (tau_s - 1/2), the
 *   interdiffusion c_S^2 (tau-_s - 1/2). */
typedef struct {
    int lattice;
    int nx, ny, nz;
    double tau_A, tau_B;
    double G;
    int precision;
    double rho_ref_A, rho_ref_B;
    double body_A;
    int forcing;
    double tau_minus_A, tau_minus_B;
} lbm_sc_params;

/* FP64 totals of one state, all reduced on the GPU in a fixed order.
 *   mass_s   = sum_x rho_s
 *   mom      = sum_x (j_A + j_B), the lattice momentum (exactly conserved)
 *   max_u    = max_x |u_phys|, u_phys = (j_A + j_B + F/2) / rho with F the
 *              total force (the F dt / 2 momentum shift of Sec. 2.3)
 *   ke       = sum_x |u_phys|^2 (the paper's kinetic-energy integral, Sec. 4.2)
 *   p_in/out = mean bulk pressure c_S^2 rho + c_S^2 G rho_A rho_B over the
 *              probe's inner ball r <= max(1, R/4) / outer region
 *              r > R + (L_min/2 - R)/2 (minimum-image r); dp = p_in - p_out;
 *              sigma = R dp in 2D (Sec. 4.1).  NaN without a probe.
 *   rhoA_in/out: mean rho_A over the same regions
 *   R_eff    = ((mass_A - rhoA_out N) / (c_d (rhoA_in - rhoA_out)))^(1/d),
 *              c_2 = pi, c_3 = 4 pi / 3
 *   n_phi_pos: number of sites with phi = rho_A - rho_B >= 0 (the droplet
 *              node count of the leakage measure, Sec. 4.2)
 *   n_nonfinite: number of sites whose rho_s or u_phys is not finite. */
typedef struct {
    double mass_A, mass_B;
    double mom[3];
    double max_u;
    double ke;
    double p_in, p_out, dp;
    double rhoA_in, rhoA_out;
    double R_eff;
    double n_in, n_out;
    double n_phi_pos;
    double n_nonfinite;
    long long step;
} lbm_sc_totals;

/* Fills *p with FP64, no body force, automatic reference densities, the
 * velocity-shift forcing and one relaxation time. */
int lbm_sc_params_default(lbm_sc_params *p, int lattice, int nx, int ny, int nz,
                          double tau_A, double tau_B, double G);

/* Device bytes a handle with these parameters needs (0 if p is invalid). */
size_t lbm_sc_bytes_needed(const lbm_sc_params *p);

/* FP64 handle that allocates its own device memory and creates its own
 * stream on the current device. */
int lbm_sc_create(lbm_sc **out, int lattice, int nx, int ny, int nz,
                  double tau_A, double tau_B, double G);

/* General constructor.  stream: a hipStream_t to enqueue on (NULL: the
 * handle creates one).  arena: caller-owned device memory of arena_bytes >=
 * lbm_sc_bytes_needed(p), 256-byte aligned (NULL: the handle allocates). */
int lbm_sc_create_ex(lbm_sc **out, const lbm_sc_params *p, void *stream, void *arena,
                     size_t arena_bytes);

/* Sets f(x, 0) = f^eq(rho_s(x), u(x)) from host arrays (u may be NULL: rest).
 * May be called again to restart.  Densities must be finite and positive
 * (LBM_EINVAL otherwise). */
int lbm_sc_init(lbm_sc *h, const double *rho_A, const double *rho_B, const double *u);

/* Enqueues n >= 0 time steps (collide, then stream).  Asynchronous. */
int lbm_sc_step(lbm_sc *h, int n);

/* Drop centre (site units) and nominal radius for the p_in / p_out / R_eff
 * totals; R <= 0 clears the probe. */
int lbm_sc_set_probe(lbm_sc *h, double cx, double cy, double cz, double R);

/* Observables of the current state, evaluated on the GPU in FP64 and copied
 * to the host.  Any pointer may be NULL.  Synchronises the stream.  Returns
 * LBM_ENONFINITE (after filling the outputs) if a density or velocity is not
 * finite. */
int lbm_sc_moments(lbm_sc *h, double *rho_A, double *rho_B, double *u, lbm_sc_totals *t);

/* Copies the population state f(x, t) to / from a host array of 2*Q*N doubles
 * (FP32_SHIFTED converts with f = h + w_i rho_ref_s).  Synchronises. */
int lbm_sc_get_populations(lbm_sc *h, double *f);
int lbm_sc_set_populations(lbm_sc *h, const double *f);

/* Blocks until the handle's queued work is done. */
int lbm_sc_sync(lbm_sc *h);

/* Enqueues n steps bracketed by two HIP events on the handle's stream, waits,
 * and returns the elapsed milliseconds of those n steps in *ms. */
int lbm_sc_time_steps(lbm_sc *h, int n, float *ms);

/* Kernel configuration.  variant: 0 = fused single-kernel step, 1 = two
 * kernels per step (densities, then collide), 2 = fused step with a
 * three-plane register pipeline (loads of plane m+2 overlap the collision of
 * plane m), 3 = fused step holding no plane across iterations (plane m is
 * pulled again, from cache, for its collision).  tx, ty: transverse
 * tile (ty = 1 on D2Q9); mb: sites marched per block along the slowest axis
 * (y on D2Q9, z on D3Q19).  Unsupported tiles return LBM_EINVAL.  A new
 * handle starts with variant 0 on D2Q9; on D3Q19 with 64 x 8 tiles (32 x 4
 * for nx <= 32), variant 0 in FP64 and 2 in FP32_SHIFTED, and march chunks
 * of about one block per compute unit.  Every configuration computes the same
 * result bit for bit. */
int lbm_sc_set_kernel(lbm_sc *h, int variant, int tx, int ty, int mb);
int lbm_sc_get_kernel(const lbm_sc *h, int *variant, int *tx, int *ty, int *mb);

/* Number of tile shapes compiled for a lattice, and the k-th one. */
int lbm_sc_tile_count(int lattice);
int lbm_sc_tile_get(int lattice, int k, int *tx, int *ty);

/* Steps applied since the last init, and the lattice parameters. */
long long lbm_sc_steps_done(const lbm_sc *h);
int lbm_sc_get_params(const lbm_sc *h, lbm_sc_params *p);

/* Device pointers of the two population buffers and the index (0/1) of the
 * one holding the current state; for zero-copy inspection only. */
int lbm_sc_device_buffers(const lbm_sc *h, void **buf0, void **buf1, int *current);

/* Layout of those buffers (either may be NULL): the array of species s and
 * velocity i starts at element (s Q + i) * stride, and site (x, y, z) sits at
 * element (z ny + y) * pitch + x of it (pitch >= nx; the elements from nx to
 * pitch of a row are padding, never read or written).  A buffer holds the
 * post-collision populations f*_is(x, t - 1) at x, so the state is read
 * pulled, f_is(x, t) = f*_is(x - c_i, t - 1) (eq. be of Sec. 2.1); elements
 * are double (LBM_FP64) or float holding f - w_i rho_ref_s (LBM_FP32_SHIFTED).
 * Lattices of 2^16 sites or more pad rows to 32 elements where the padded
 * arrays keep 32-bit byte offsets.  LBM_EINVAL for a NULL handle. */
int lbm_sc_buffer_layout(const lbm_sc *h, size_t *stride, int *pitch);

/* Releases the handle (NULL is a no-op).  Waits for its queued work. */
int lbm_sc_destroy(lbm_sc *h);

const char *lbm_sc_strerror(int status);

/* Streaming-copy ceiling on this device: reads and writes nbytes of device
 * memory once with the same load/store width as the step kernels and returns
 * the kernel's elapsed milliseconds (averaged over reps launches).  src and
 * dst are caller-owned device buffers of at least nbytes.  Used to report the
 * achievable HBM bandwidth beside the step's roofline fraction. */
int lbm_sc_copy_bench(void *dst, const void *src, size_t nbytes, int reps, void *stream,
                      float *ms);

/* ---------------------------------------------------------------------------
 * Batched execution: many independent lattices advanced together.
 *
 * Handles joined to a batch keep their own state and parameters; the batch
 * advances every member with steps remaining by up to epoch_steps steps per
 * run call.  Per-site arithmetic is the same code as lbm_sc_step(), so a
 * lattice evolves bitwise the same alone or inside a batch.
 * ------------------------------------------------------------------------- */

/* mode for lbm_batch_run */
enum {
    LBM_BATCH_PER_LATTICE = 0, /* one launch per lattice per step (baseline) */
    LBM_BATCH_FUSED = 1,       /* one launch per lattice group per step, all lattices
                                  (graph-replayed; the fastest form measured) */
    LBM_BATCH_PERSISTENT = 2   /* one persistent launch per epoch with grid barriers
                                  (for callers that want one launch per epoch) */
};

/* hbm_budget: bytes of member state the batch admits (0: unlimited).
 * stream: hipStream_t to run on (NULL: the batch creates one). */
int lbm_batch_create(lbm_batch **out, size_t hbm_budget, void *stream);

/* Adds an initialised handle with `steps` steps to run.  LBM_EBUDGET when its
 * bytes exceed the remaining budget; LBM_EINVAL for a handle already in a
 * batch.  The batch does not own the handle. */
int lbm_batch_add(lbm_batch *b, lbm_sc *h, long long steps);

/* Removes a member (finished or not).  The handle stays valid.  Waits for the
 * batch's stream; returns LBM_ETIMEOUT (after removing the member) if a
 * persistent launch of the batch gave up at a grid barrier (see
 * lbm_batch_poll). */
int lbm_batch_remove(lbm_batch *b, lbm_sc *h);

/* Enqueues up to epoch_steps steps of every member with steps remaining.
 * Asynchronous; graph-captured where the mode allows. */
int lbm_batch_run(lbm_batch *b, int epoch_steps, int mode);

/* Allocation-free variant of lbm_batch_run, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  No device memory is allocated and no graph is
 * built: the fused form's descriptor table and work list are copied into a
 * fixed device array of the library (about 4.5 MB, one per GPU, held until
 * the process ends) and the epoch is launched directly, one kernel per step.
 * Limits per kernel policy group (precision x forcing x relaxation):
 * 1024 members and 262144 work items (tiles x march chunks); beyond them the
 * call returns LBM_ETOOBIG before enqueueing anything.
 * mode: LBM_BATCH_FUSED, or LBM_BATCH_PER_LATTICE (which uses no tables and
 * runs as lbm_batch_run does); LBM_BATCH_PERSISTENT returns LBM_EINVAL.
 * Results are bitwise those of lbm_batch_run (the same kernels).
 * Every call on a GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (from several batches or threads, on different
 * streams) race and must be serialised by the caller.  The host-side tables
 * are staged in memory the batch keeps; each call waits for the previous
 * upload of its batch before reusing it. */
int lbm_batch_run_noalloc(lbm_batch *b, int epoch_steps, int mode);

/* Waits for the batch's stream, then writes up to max_done members whose
 * steps are complete into done[] and their count into *n_done (finished
 * members stay in the batch until removed).  Returns LBM_ETIMEOUT if a
 * persistent launch gave up at a grid barrier (its blocks waited longer than
 * the spin limit for the others, e.g. because they were not co-resident):
 * every block then leaves the kernel, the members are left part way through
 * the epoch, the batch is failed and each member handle accepts only removal
 * and lbm_sc_destroy.  The flag that reports it survives later launches until
 * the host has read it here, in lbm_batch_remove or in lbm_batch_destroy. */
int lbm_batch_poll(lbm_batch *b, lbm_sc **done, int max_done, int *n_done);

/* Members, bytes in use and pending site-updates of the batch. */
int lbm_batch_stats(const lbm_batch *b, int *members, size_t *bytes_used,
                    double *pending_site_updates);

/* Sets the transverse tile used for each lattice type inside fused and
 * persistent batch launches (0 keeps the default). */
int lbm_batch_set_tiles(lbm_batch *b, int tx9, int tx19, int ty19, int mb9, int mb19);

/* Grid-barrier polls (each a short sleep) a block of a persistent launch
 * makes before it gives up and the launch reports LBM_ETIMEOUT; 0 restores
 * the default (2^26, seconds).  A small value forces the give-up path. */
int lbm_batch_set_spin_limit(lbm_batch *b, unsigned spins);

/* Releases the batch (its members stay valid and leave it).  Waits for its
 * stream; returns LBM_ETIMEOUT if an unreported persistent-launch give-up is
 * found, LBM_OK otherwise. */
int lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SC_H */
