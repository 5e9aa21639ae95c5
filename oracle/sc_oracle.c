/*
 * sc_oracle.c -- plain, slow, FP64 CPU oracle of the two-component Shan-Chen
 * BGK lattice Boltzmann time step.
 *
 *   Scarbolo, Molin, Perlekar, Sbragaglia, Soldati, Toschi, "Unified framework
 *   for a side-by-side comparison of different multicomponent algorithms:
 *   lattice Boltzmann vs. phase field model", Sec. 2.1.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the HIP library
 * against the paper.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it; the library itself never calls it.
 * It shares no code, header, table or constant with the HIP path.
 *
 * Everything is written the slow and obvious way: one loop per step of the
 * method, in the paper's order and notation, double precision throughout, no
 * blocking or fusion.  Built with -O2 -ffp-contract=off (no fused multiply-add,
 * no fast-math).  The per-site loops carry OpenMP pragmas: the default build
 * ignores them (one thread); the all-core build used only to time the oracle
 * on the host runs the same per-site arithmetic, with the sites of a loop
 * shared out among threads (no reductions, so the results are bitwise equal).
 *
 * Layout of a population array f: f[s][i][z][y][x], x fastest, species s in
 * {A=0, B=1}, velocity i in [0, Q).  N = nx*ny*nz sites.  The state held
 * between steps is the post-streaming (pre-collision) f(x, t).
 *
 * Parity status: every function here is pinned by the CPU tests (isotropy
 * sums, equilibrium moments, streaming permutation, closed-form force gather,
 * conservation laws, fixed points, shear-wave and interdiffusion decay rates,
 * the linearised Fourier-mode update, the continuum growth rate of the
 * paper's chemical potential, the worked example's bulk order parameter and
 * Laplace-law linearity; for the Guo forcing option: exact mass and
 * momentum balance, the laminar Kolmogorov profile, and the linearised growth
 * rate with the bare coupling g in place of g^(tau); for two relaxation
 * times: the BGK limit, nu from the even and D from the odd relaxation time,
 * the linearised update and its growth-rate limit), and cross-checked
 * against an independent NumPy implementation on small grids.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* c_S^2 = 1/3 (Sec. 2.1, the constant in the weight normalisation). */
static const double CS2 = 1.0 / 3.0;

/* ---------------------------------------------------------------------------
 * Velocity sets.  The paper does not print D2Q9/D3Q19; it fixes the weights
 * by their normalisation: sum_i w_i c_ia c_ib = c_S^2 delta_ab and the
 * fourth-order isotropy sum = c_S^4 (dd + dd + dd) (Sec. 2.1).  These are the
 * standard sets satisfying both, listed in the library's export order.
 * ------------------------------------------------------------------------- */
static const int C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {
    4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int C19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, -1}, {0, 1, 1}, {0, -1, -1},
    {1, -1, 0}, {-1, 1, 0}, {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
    int q;
    int nx, ny, nz;
    long n;
    const int (*c)[3];
    const double *w;
} lat_t;

static int lat_make(lat_t *L, int q, int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    if (q == 9) {
        if (nz != 1) return -1;
        L->c = C9;
        L->w = W9;
    } else if (q == 19) {
        L->c = C19;
        L->w = W19;
    } else {
        return -1;
    }
    L->q = q;
    L->nx = nx;
    L->ny = ny;
    L->nz = nz;
    L->n = (long)nx * ny * nz;
    return 0;
}

static long wrap(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

/* Site index of (x + dx, y + dy, z + dz) on the periodic lattice. */
static long site_shift(const lat_t *L, long x, long y, long z, int dx, int dy, int dz) {
    long xx = wrap(x + dx, L->nx), yy = wrap(y + dy, L->ny), zz = wrap(z + dz, L->nz);
    return (zz * L->ny + yy) * L->nx + xx;
}

/* f[s][i][site] */
static long fidx(const lat_t *L, int s, int i, long site) {
    return ((long)s * L->q + i) * L->n + site;
}

int oracle_lattice(int q, int *c_out, double *w_out) {
    lat_t L;
    if (lat_make(&L, q, 1, 1, 1) != 0) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = L.c[i][a];
        w_out[i] = L.w[i];
    }
    return 0;
}

/* Local Maxwellian truncated at second order (Sec. 2.1, the equilibrium of
 * eq:be), the standard Hermite form with c_S^2 = 1/3:
 *   f_i^eq(rho, v) = w_i rho [1 + c_i.v / c_S^2 + (c_i.v)^2 / (2 c_S^4) - v.v / (2 c_S^2)]. */
static void feq_at(const lat_t *L, double rho, const double v[3], double *feq) {
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int i = 0; i < L->q; ++i) {
        double cv = L->c[i][0] * v[0] + L->c[i][1] * v[1] + L->c[i][2] * v[2];
        feq[i] = L->w[i] * rho *
                 (1.0 + cv / CS2 + (cv * cv) / (2.0 * CS2 * CS2) - vv / (2.0 * CS2));
    }
}

int oracle_feq(int q, double rho, const double *v, double *feq) {
    lat_t L;
    if (lat_make(&L, q, 1, 1, 1) != 0) return -1;
    feq_at(&L, rho, v, feq);
    return 0;
}

/* Initial populations: the equilibrium at the given densities and velocity
 * (u = 0 when u is NULL).  The paper does not state how f(x, 0) is chosen. */
int oracle_init(int q, int nx, int ny, int nz, const double *rhoA, const double *rhoB,
                const double *u, double *f) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    const double *rho[2] = {rhoA, rhoB};
    double feq[19];
    for (long x = 0; x < L.n; ++x) {
        double v[3] = {0.0, 0.0, 0.0};
        if (u) {
            v[0] = u[x];
            v[1] = u[L.n + x];
            v[2] = u[2 * L.n + x];
        }
        for (int s = 0; s < 2; ++s) {
            feq_at(&L, rho[s][x], v, feq);
            for (int i = 0; i < q; ++i) f[fidx(&L, s, i, x)] = feq[i];
        }
    }
    return 0;
}

/* Species densities and momenta: rho_s = sum_i f_is, j_s = sum_i f_is c_i
 * (Sec. 2.1, the moment definitions below eq:be).
 * rho[s*N + x], j[(s*3 + a)*N + x]. */
int oracle_moments(int q, int nx, int ny, int nz, const double *f, double *rho, double *j) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    for (int s = 0; s < 2; ++s) {
#pragma omp parallel for schedule(static)
        for (long x = 0; x < L.n; ++x) {
            double r = 0.0, ja[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < q; ++i) {
                double fi = f[fidx(&L, s, i, x)];
                r += fi;
                for (int a = 0; a < 3; ++a) ja[a] += fi * L.c[i][a];
            }
            rho[s * L.n + x] = r;
            if (j)
                for (int a = 0; a < 3; ++a) j[(s * 3 + a) * L.n + x] = ja[a];
        }
    }
    return 0;
}

/* Inter-species Shan-Chen force, eq. FORCE with psi = rho, a symmetric
 * coupling G_AB = G_BA = G and no self-interaction:
 *   F_s(x) = -G rho_s(x) sum_i w_i rho_s'(x + c_i) c_i,  s' != s.
 * F[(s*3 + a)*N + x]. */
int oracle_force(int q, int nx, int ny, int nz, double G, const double *rho, double *F) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long site = ((long)z * ny + y) * nx + x;
                for (int s = 0; s < 2; ++s) {
                    int so = 1 - s;
                    double sum[3] = {0.0, 0.0, 0.0};
                    for (int i = 0; i < q; ++i) {
                        long nb = site_shift(&L, x, y, z, L.c[i][0], L.c[i][1], L.c[i][2]);
                        double r = rho[so * L.n + nb];
                        for (int a = 0; a < 3; ++a) sum[a] += L.w[i] * r * L.c[i][a];
                    }
                    for (int a = 0; a < 3; ++a)
                        F[(s * 3 + a) * L.n + site] = -G * rho[s * L.n + site] * sum[a];
                }
            }
    return 0;
}

/* Optional Kolmogorov body force of the paper's sheared-drop test (Sec. 4.2):
 * F_x = rho_s A sin(2 pi y / L_y), added to each species' force. */
static double kolmogorov(double A, int y, int ny) {
    return A * sin(2.0 * M_PI * (double)y / (double)ny);
}

/* Forcing schemes.  ORACLE_FORCING_SHIFT is the paper's (Sec. 2.1): the
 * force enters only through the shifted equilibrium velocity v_s.
 * ORACLE_FORCING_GUO is the discrete forcing of Guo, Zheng and Shi (2002),
 * which the paper cites as the way to remove the tau-dependence of the
 * effective coupling g^(tau) = tau g / (tau - 1/2) (Sec. 2.3).  The paper
 * gives no formula for it; this is the standard form applied per species:
 *   u      = sum_s (j_s + F_s / 2) / tau_s  /  sum_s rho_s / tau_s
 *   f*_is  = f_is - (f_is - f^eq_is(rho_s, u)) / tau_s + S_is
 *   S_is   = (1 - 1 / (2 tau_s)) w_i [ (c_i - u).F_s / c_S^2
 *                                      + (c_i.u)(c_i.F_s) / c_S^4 ]
 * Sum_i S_is = 0 and sum_i S_is c_i = (1 - 1/(2 tau_s)) F_s, so the step
 * conserves each species' mass and adds exactly sum_s F_s of momentum. */
enum { ORACLE_FORCING_SHIFT = 0, ORACLE_FORCING_GUO = 1 };

static double guo_source(const lat_t *L, int i, const double u[3], const double F[3],
                         double tau) {
    double cu = 0.0, cF = 0.0, uF = 0.0;
    for (int a = 0; a < 3; ++a) {
        cu += L->c[i][a] * u[a];
        cF += L->c[i][a] * F[a];
        uF += u[a] * F[a];
    }
    return (1.0 - 1.0 / (2.0 * tau)) * L->w[i] * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2));
}

/* Index of the velocity opposite to c_i. */
static int opposite(const lat_t *L, int i) {
    for (int k = 0; k < L->q; ++k)
        if (L->c[k][0] == -L->c[i][0] && L->c[k][1] == -L->c[i][1] && L->c[k][2] == -L->c[i][2])
            return k;
    return i;
}

/* Collision of the populations fin[s*Q + i] of one site into fout, given the
 * moments rho_s, j_s and the total force F_s (body force included) of both
 * species.
 *
 * taup_s is the BGK relaxation time tau_s of eq:be.  taum_s is the relaxation
 * time of the odd (antisymmetric) part of the populations: equal to taup_s
 * the collision is the paper's BGK; different, it is the two-relaxation-time
 * member of the multiple-relaxation-time family the paper cites (Sec. 2.1,
 * last paragraph) for decoupling the diffusive and viscous time scales:
 *   f*_i = f_i - (f+_i - feq+_i) / taup - (f-_i - feq-_i) / taum,
 *   f+-_i = (f_i +- f_ibar) / 2,  ibar the velocity opposite to i.
 * The odd moments carry the species momenta, so the momentum exchange and the
 * force shift use taum: u' = sum_s j_s / taum_s / sum_s rho_s / taum_s and
 * v_s = u' + taum_s F_s / rho_s.  The even moments carry the stress, so the
 * viscosity is c_S^2 (taup - 1/2) and the interdiffusion c_S^2 (taum - 1/2).
 * With Guo forcing the source splits likewise: its even part
 * w_i [9 (c_i.u)(c_i.F_s) - 3 u.F_s] takes (1 - 1/(2 taup)), its odd part
 * w_i 3 c_i.F_s takes (1 - 1/(2 taum)). */
static void collide_site(const lat_t *L, const double rho[2], const double j[2][3],
                         const double F[2][3], const double taup[2], const double taum[2],
                         int forcing, const double *fin, double *fout) {
    const int q = L->q;
    double u[3], num[3] = {0.0, 0.0, 0.0}, den = 0.0;
    for (int s = 0; s < 2; ++s) {
        for (int a = 0; a < 3; ++a)
            num[a] += (forcing == ORACLE_FORCING_GUO ? j[s][a] + 0.5 * F[s][a] : j[s][a]) / taum[s];
        den += rho[s] / taum[s];
    }
    for (int a = 0; a < 3; ++a) u[a] = num[a] / den;
    for (int s = 0; s < 2; ++s) {
        double v[3], feq[19];
        for (int a = 0; a < 3; ++a)
            v[a] = forcing == ORACLE_FORCING_GUO ? u[a] : u[a] + taum[s] * F[s][a] / rho[s];
        feq_at(L, rho[s], v, feq);
        for (int i = 0; i < q; ++i) {
            double fi = fin[s * q + i], out;
            if (taum[s] == taup[s]) {
                out = fi - (fi - feq[i]) / taup[s];
                if (forcing == ORACLE_FORCING_GUO) out += guo_source(L, i, u, F[s], taup[s]);
            } else {
                int ib = opposite(L, i);
                double fb = fin[s * q + ib];
                double fp = 0.5 * (fi + fb), fm = 0.5 * (fi - fb);
                double ep = 0.5 * (feq[i] + feq[ib]), em = 0.5 * (feq[i] - feq[ib]);
                out = fi - (fp - ep) / taup[s] - (fm - em) / taum[s];
                if (forcing == ORACLE_FORCING_GUO) {
                    double cu = 0.0, cF = 0.0, uF = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        cu += L->c[i][a] * u[a];
                        cF += L->c[i][a] * F[s][a];
                        uF += u[a] * F[s][a];
                    }
                    double even = L->w[i] * (cu * cF / (CS2 * CS2) - uF / CS2);
                    double odd = L->w[i] * cF / CS2;
                    out += (1.0 - 1.0 / (2.0 * taup[s])) * even + (1.0 - 1.0 / (2.0 * taum[s])) * odd;
                }
            }
            fout[s * q + i] = out;
        }
    }
}

/* One BGK collision of both species (eq:be, right-hand side).  Velocity
 * shift (the paper's scheme):
 *   u    = sum_s (1/tau_s) j_s / sum_s (1/tau_s) rho_s       (common velocity)
 *   v_s  = u + tau_s F_s / rho_s                              (force shift)
 *   f*_is = f_is - (f_is - f_is^eq(rho_s, v_s)) / tau_s;
 * Guo forcing as described above.  fpost may not alias f. */
int oracle_collide(int q, int nx, int ny, int nz, double tauA, double tauB, double G,
                   double bodyA, const double *f, double *fpost, int forcing, double tmA,
                   double tmB) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    double *rho = malloc(sizeof(double) * 2 * L.n);
    double *j = malloc(sizeof(double) * 6 * L.n);
    double *F = malloc(sizeof(double) * 6 * L.n);
    if (!rho || !j || !F) {
        free(rho);
        free(j);
        free(F);
        return -2;
    }
    oracle_moments(q, nx, ny, nz, f, rho, j);
    oracle_force(q, nx, ny, nz, G, rho, F); /* psi_s = rho_s */
    const double taup[2] = {tauA, tauB};
    const double taum[2] = {tmA > 0.0 ? tmA : tauA, tmB > 0.0 ? tmB : tauB};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long site = ((long)z * ny + y) * nx + x;
                double fin[38], fout[38];
                double r[2], js[2][3], Fs[2][3];
                for (int s = 0; s < 2; ++s) {
                    r[s] = rho[s * L.n + site];
                    for (int a = 0; a < 3; ++a) {
                        js[s][a] = j[(s * 3 + a) * L.n + site];
                        Fs[s][a] = F[(s * 3 + a) * L.n + site];
                    }
                    if (bodyA != 0.0) Fs[s][0] += r[s] * kolmogorov(bodyA, y, ny);
                    for (int i = 0; i < q; ++i) fin[s * q + i] = f[fidx(&L, s, i, site)];
                }
                collide_site(&L, r, js, Fs, taup, taum, forcing, fin, fout);
                for (int s = 0; s < 2; ++s)
                    for (int i = 0; i < q; ++i) fpost[fidx(&L, s, i, site)] = fout[s * q + i];
            }
    free(rho);
    free(j);
    free(F);
    return 0;
}

/* Free streaming (eq:be, left-hand side, Delta t = 1) on the periodic lattice:
 *   f_is(x + c_i, t + 1) = f*_is(x, t).  fnew may not alias fpost. */
int oracle_stream(int q, int nx, int ny, int nz, const double *fpost, double *fnew) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < q; ++i)
#pragma omp parallel for schedule(static)
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        long site = ((long)z * ny + y) * nx + x;
                        long dest = site_shift(&L, x, y, z, L.c[i][0], L.c[i][1], L.c[i][2]);
                        fnew[fidx(&L, s, i, dest)] = fpost[fidx(&L, s, i, site)];
                    }
    return 0;
}

/* nsteps full time steps (collide, then stream), in place on f. */
int oracle_run(int q, int nx, int ny, int nz, double tauA, double tauB, double G,
               double bodyA, double *f, int nsteps, int forcing, double tmA, double tmB) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0 || nsteps < 0) return -1;
    double *tmp = malloc(sizeof(double) * 2 * q * L.n);
    if (!tmp) return -2;
    for (int t = 0; t < nsteps; ++t) {
        oracle_collide(q, nx, ny, nz, tauA, tauB, G, bodyA, f, tmp, forcing, tmA, tmB);
        oracle_stream(q, nx, ny, nz, tmp, f);
    }
    free(tmp);
    return 0;
}

/* Observables of the state f(x, t), all FP64.
 *
 *   rho_out[2N]   : rho_A, rho_B
 *   u_out[3N]     : u_phys = (sum_s j_s + F/2) / rho with F = sum_s F_s, the
 *                   lattice momentum shifted by F dt / 2 (Sec. 2.3) over the
 *                   total density rho = rho_A + rho_B (Sec. 2.1)
 *   p_out[N]      : bulk pressure c_S^2 (rho_A + rho_B) + c_S^2 G rho_A rho_B
 *                   (Sec. 2.1, the isotropic part of the SC pressure tensor
 *                   without gradient terms)
 *   totals[16]    : see OT_* below.
 * probe = {cx, cy, cz, R} or NULL: the drop centre and nominal radius used for
 * the inside/outside pressure means and R_eff; any output may be NULL. */
enum {
    OT_MASS_A, OT_MASS_B, OT_MOM_X, OT_MOM_Y, OT_MOM_Z, OT_MAX_U, OT_P_IN, OT_P_OUT,
    OT_DP, OT_R_EFF, OT_N_PHI_POS, OT_KE, OT_RHOA_IN, OT_RHOA_OUT, OT_N_IN, OT_N_OUT,
    OT_COUNT
};

int oracle_observables(int q, int nx, int ny, int nz, double tauA, double tauB, double G,
                       double bodyA, const double *f, const double *probe, double *rho_out,
                       double *u_out, double *p_out, double *totals) {
    (void)tauA;
    (void)tauB;
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    double *rho = malloc(sizeof(double) * 2 * L.n);
    double *j = malloc(sizeof(double) * 6 * L.n);
    double *F = malloc(sizeof(double) * 6 * L.n);
    if (!rho || !j || !F) {
        free(rho);
        free(j);
        free(F);
        return -2;
    }
    oracle_moments(q, nx, ny, nz, f, rho, j);
    oracle_force(q, nx, ny, nz, G, rho, F);
    double T[OT_COUNT];
    for (int k = 0; k < OT_COUNT; ++k) T[k] = 0.0;
    double r_in = 0.0, r_out = 0.0;
    if (probe) {
        double R = probe[3];
        double half = 0.5 * (nx < ny ? nx : ny);
        if (nz > 1 && 0.5 * nz < half) half = 0.5 * nz;
        r_in = R / 4.0 > 1.0 ? R / 4.0 : 1.0;
        r_out = R + 0.5 * (half - R);
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long site = ((long)z * ny + y) * nx + x;
                double rA = rho[site], rB = rho[L.n + site];
                double r = rA + rB;
                double u[3];
                for (int a = 0; a < 3; ++a) {
                    double Ft = F[a * L.n + site] + F[(3 + a) * L.n + site];
                    if (a == 0 && bodyA != 0.0) Ft += r * kolmogorov(bodyA, y, ny);
                    double mom = j[a * L.n + site] + j[(3 + a) * L.n + site];
                    u[a] = (mom + 0.5 * Ft) / r;
                    T[OT_MOM_X + a] += mom;
                }
                double umag = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double p = CS2 * (rA + rB) + CS2 * G * rA * rB;
                T[OT_MASS_A] += rA;
                T[OT_MASS_B] += rB;
                if (umag > T[OT_MAX_U]) T[OT_MAX_U] = umag;
                T[OT_KE] += u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                if (rA - rB >= 0.0) T[OT_N_PHI_POS] += 1.0;
                if (probe) {
                    double dx = x - probe[0], dy = y - probe[1], dz = z - probe[2];
                    dx -= nx * round(dx / nx);
                    dy -= ny * round(dy / ny);
                    dz = nz > 1 ? dz - nz * round(dz / nz) : 0.0;
                    double d = sqrt(dx * dx + dy * dy + dz * dz);
                    if (d <= r_in) {
                        T[OT_P_IN] += p;
                        T[OT_RHOA_IN] += rA;
                        T[OT_N_IN] += 1.0;
                    } else if (d > r_out) {
                        T[OT_P_OUT] += p;
                        T[OT_RHOA_OUT] += rA;
                        T[OT_N_OUT] += 1.0;
                    }
                }
                if (rho_out) {
                    rho_out[site] = rA;
                    rho_out[L.n + site] = rB;
                }
                if (u_out)
                    for (int a = 0; a < 3; ++a) u_out[a * L.n + site] = u[a];
                if (p_out) p_out[site] = p;
            }
    if (probe && T[OT_N_IN] > 0 && T[OT_N_OUT] > 0) {
        T[OT_P_IN] /= T[OT_N_IN];
        T[OT_P_OUT] /= T[OT_N_OUT];
        T[OT_RHOA_IN] /= T[OT_N_IN];
        T[OT_RHOA_OUT] /= T[OT_N_OUT];
        T[OT_DP] = T[OT_P_IN] - T[OT_P_OUT];
        /* Effective radius from the species-A mass excess over the outer bulk:
         * c_d R^d (rho_in - rho_out) = M_A - rho_out V, c_2 = pi, c_3 = 4 pi / 3. */
        int d = nz > 1 ? 3 : 2;
        double cd = d == 3 ? 4.0 * M_PI / 3.0 : M_PI;
        double vol = (double)L.n;
        double num = T[OT_MASS_A] - T[OT_RHOA_OUT] * vol;
        double den = cd * (T[OT_RHOA_IN] - T[OT_RHOA_OUT]);
        T[OT_R_EFF] = pow(num / den, 1.0 / d);
    } else {
        T[OT_P_IN] = T[OT_P_OUT] = T[OT_DP] = T[OT_R_EFF] = NAN;
        T[OT_RHOA_IN] = T[OT_RHOA_OUT] = NAN;
    }
    if (totals)
        for (int k = 0; k < OT_COUNT; ++k) totals[k] = T[k];
    free(rho);
    free(j);
    free(F);
    return 0;
}

/* Post-step populations at selected sites only, computed one by one from the
 * full state f(x, t): f_is(x, t+1) = f*_is(x - c_i, t) (pull form of the same
 * streaming).  out[k*2Q + s*Q + i] for site sites[k].  Used to check large
 * lattices where a full oracle step is too slow to run in a test. */
int oracle_step_sites(int q, int nx, int ny, int nz, double tauA, double tauB, double G,
                      double bodyA, const double *f, const long *sites, int nsites,
                      double *out, int forcing, double tmA, double tmB) {
    lat_t L;
    if (lat_make(&L, q, nx, ny, nz) != 0) return -1;
    const double taup[2] = {tauA, tauB};
    const double taum[2] = {tmA > 0.0 ? tmA : tauA, tmB > 0.0 ? tmB : tauB};
    double fin[38], fout[38];
    for (int k = 0; k < nsites; ++k) {
        long site = sites[k];
        if (site < 0 || site >= L.n) return -1;
        int x = (int)(site % nx), y = (int)((site / nx) % ny), z = (int)(site / ((long)nx * ny));
        for (int i = 0; i < q; ++i) {
            /* the upstream site y0 = x - c_i collides, then its f*_i streams here */
            int x0 = (int)wrap(x - L.c[i][0], nx), y0 = (int)wrap(y - L.c[i][1], ny),
                z0 = (int)wrap(z - L.c[i][2], nz);
            long up = ((long)z0 * ny + y0) * nx + x0;
            double rho[2], j[2][3];
            for (int s = 0; s < 2; ++s) {
                rho[s] = 0.0;
                j[s][0] = j[s][1] = j[s][2] = 0.0;
                for (int k2 = 0; k2 < q; ++k2) {
                    double fv = f[fidx(&L, s, k2, up)];
                    rho[s] += fv;
                    for (int a = 0; a < 3; ++a) j[s][a] += fv * L.c[k2][a];
                    fin[s * q + k2] = fv;
                }
            }
            double Fs[2][3];
            for (int s = 0; s < 2; ++s) {
                int so = 1 - s;
                double sum[3] = {0.0, 0.0, 0.0};
                for (int k2 = 0; k2 < q; ++k2) {
                    long nb = site_shift(&L, x0, y0, z0, L.c[k2][0], L.c[k2][1], L.c[k2][2]);
                    double r = 0.0;
                    for (int k3 = 0; k3 < q; ++k3) r += f[fidx(&L, so, k3, nb)];
                    for (int a = 0; a < 3; ++a) sum[a] += L.w[k2] * r * L.c[k2][a];
                }
                for (int a = 0; a < 3; ++a) Fs[s][a] = -G * rho[s] * sum[a];
                if (bodyA != 0.0) Fs[s][0] += rho[s] * kolmogorov(bodyA, y0, ny);
            }
            collide_site(&L, rho, j, Fs, taup, taum, forcing, fin, fout);
            for (int s = 0; s < 2; ++s) out[(long)k * 2 * q + s * q + i] = fout[s * q + i];
        }
    }
    return 0;
}
