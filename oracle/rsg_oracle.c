/*
 * rsg_oracle.c -- plain FP64 reference ("oracle") for the real-space
 * Kohn-Sham H*psi / Taylor-propagation path.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark load this file.  The GPU library neither
 * links nor calls it, and this file shares no code, header or table with
 * the GPU library.
 *
 * Everything below is the definition written out as plain loops in double /
 * double complex, in the order the definition states: no blocking, no
 * fusion, no reordering.  OpenMP is used only over independent output
 * points of H*psi, where each output is still computed by exactly one
 * thread in the same tap order; every reduction is a single serial sum in
 * compact point order.
 *
 * What follows the paper, and where the paper is silent:
 *  - Uniform real-space grid; integrals become grid sums with weight h^3 and
 *    differential operators become high-order finite differences (section
 *    "Introduction").  The order is not given there: this is the 8th-order
 *    25-point star (centred second-derivative weights of Fornberg 1988,
 *    c0..c4 = -205/72, 8/5, -1/5, 8/315, -1/560).
 *  - Fields are linear arrays over the points of the simulation box plus
 *    separate grid metadata; the box here is a sphere or a cube (section
 *    "Parallelization, optimizations and graphics processing units").
 *    Orbitals outside the box are zero (Dirichlet; the paper is silent).
 *  - Kinetic term -1/2 Laplacian in atomic units; the prefactor is a
 *    parameter so that tests can switch the kinetic term off.
 *  - Non-local pseudopotential in separable (Kleinman-Bylander) form:
 *    V_nl psi = sum_a sum_i p_i^a E_i^a <p_i^a|psi>, real projectors.  The
 *    paper names the non-local potential and its projectors (section
 *    "Magnetic response and gauge invariance in real-space grids") but not
 *    their form.
 *  - Dipole coupling E(t) * x_axis to the control field (section
 *    "Quantum optimal control": the handle is a time-dependent electric
 *    field whose parameters are Fourier coefficients of its amplitude).
 *  - Discrete evolution operator U(dt) applied recursively (section
 *    "Photoemission"); realised as the 4th-order Taylor expansion of
 *    exp(-i dt H), with H evaluated at the step midpoint.  The same section's
 *    mask boundary absorber multiplies each propagated orbital by a real mask
 *    M(r) after every step (eq. (mask_split)); M itself is an input (the
 *    paper gives no formula for it).
 *  - Optimal-control gradient, eq. (qoctgradient), with the costate
 *    propagated backwards by the adjoint of the forward propagator.  The
 *    oracle computes the exact gradient of the time-discretised target
 *    (discrete adjoint); the continuous formula is its dt -> 0 limit.
 *  - Complex scaling r -> r e^{i theta} (section "Complex scaling and
 *    resonances"): the kinetic prefactor becomes kin e^{-2 i theta} and the
 *    local potential its analytic continuation v(r e^{i theta}), whose real
 *    and imaginary parts are inputs; the operator stays symmetric (not
 *    Hermitian), and its matrix elements take no complex conjugation.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int32_t n[3];        /* tight bounding box (x, y, z) */
    int64_t np;          /* number of points in the simulation box */
    double h;            /* grid spacing (bohr) */
    const int32_t *ijk;  /* [np][3] box coordinates, 0 <= ijk[a] < n[a] */
    const int64_t *map;  /* [n2][n1][n0]: compact index, or -1 outside */
} or_grid;

typedef struct {
    const double *V;         /* [np] local potential (Hartree) */
    double kin;              /* kinetic prefactor: -0.5 for -1/2 Laplacian */
    int32_t dipole_axis;     /* 0, 1, 2, or -1 for no dipole coupling */
    int32_t natoms;
    const int64_t *kb_off;   /* [natoms+1] offsets into kb_idx and kb_p */
    const int32_t *kb_idx;   /* compact indices of every support S_a */
    const double *kb_p;      /* [entries][4] projector values */
    const double *kb_E;      /* [natoms][4] projector energies */
    double kin_im;           /* imaginary part of the kinetic prefactor (complex scaling) */
    const double *V_im;      /* [np] imaginary part of the local potential, or NULL */
} or_ham;

/* ---------------------------------------------------------------------- */
/* Grid: sphere or cube, compact order z-major, then y, then x.            */
/* ---------------------------------------------------------------------- */

static int64_t sphere_q(double R, double h) { return (int64_t)floor((R / h) * (R / h) + 1e-9); }

static int64_t isqrt64(int64_t q) {
    int64_t m = (int64_t)sqrt((double)q);
    while ((m + 1) * (m + 1) <= q) ++m;
    while (m * m > q) --m;
    return m;
}

/* Sphere centred on a grid point: centred integer offsets (i, j, k) are in
   the box iff i^2 + j^2 + k^2 <= floor((R/h)^2 + 1e-9).  Returns np and the
   tight box size in dims[3]; writes [np][3] coordinates if ijk != NULL. */
int64_t or_sphere_points(double R, double h, int32_t *dims, int32_t *ijk) {
    const int64_t q = sphere_q(R, h);
    const int64_t m = isqrt64(q);
    int64_t np = 0;
    for (int64_t k = -m; k <= m; ++k)
        for (int64_t j = -m; j <= m; ++j)
            for (int64_t i = -m; i <= m; ++i)
                if (i * i + j * j + k * k <= q) {
                    if (ijk) {
                        ijk[3 * np + 0] = (int32_t)(i + m);
                        ijk[3 * np + 1] = (int32_t)(j + m);
                        ijk[3 * np + 2] = (int32_t)(k + m);
                    }
                    ++np;
                }
    if (dims) dims[0] = dims[1] = dims[2] = (int32_t)(2 * m + 1);
    return np;
}

/* Rectangular box of nx x ny x nz points (every point of the tight box). */
int64_t or_box_points(int32_t nx, int32_t ny, int32_t nz, int32_t *dims, int32_t *ijk) {
    int64_t np = 0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                if (ijk) {
                    ijk[3 * np + 0] = i;
                    ijk[3 * np + 1] = j;
                    ijk[3 * np + 2] = k;
                }
                ++np;
            }
    if (dims) {
        dims[0] = nx;
        dims[1] = ny;
        dims[2] = nz;
    }
    return np;
}

/* Cube of n points per axis. */
int64_t or_cube_points(int32_t n, int32_t *dims, int32_t *ijk) { return or_box_points(n, n, n, dims, ijk); }

/* Dense index map over the tight box. */
void or_index_map(const int32_t *dims, int64_t np, const int32_t *ijk, int64_t *map) {
    const int64_t total = (int64_t)dims[0] * dims[1] * dims[2];
    for (int64_t c = 0; c < total; ++c) map[c] = -1;
    for (int64_t p = 0; p < np; ++p) {
        const int32_t *c = ijk + 3 * p;
        map[((int64_t)c[2] * dims[1] + c[1]) * dims[0] + c[0]] = p;
    }
}

/* Position along one axis: x_a = h (ijk_a - (n_a - 1)/2); the box is
   symmetric about the origin. */
static double coord(const or_grid *g, int64_t p, int axis) {
    return g->h * ((double)g->ijk[3 * p + axis] - 0.5 * (double)(g->n[axis] - 1));
}

void or_positions(const or_grid *g, double *xyz) {
    for (int64_t p = 0; p < g->np; ++p)
        for (int a = 0; a < 3; ++a) xyz[3 * p + a] = coord(g, p, a);
}

static int64_t lookup(const or_grid *g, int32_t x, int32_t y, int32_t z) {
    if (x < 0 || y < 0 || z < 0 || x >= g->n[0] || y >= g->n[1] || z >= g->n[2]) return -1;
    return g->map[((int64_t)z * g->n[1] + y) * g->n[0] + x];
}

/* ---------------------------------------------------------------------- */
/* H psi                                                                   */
/* ---------------------------------------------------------------------- */

static const double FD8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

/* out = H psi, with
     (H psi)(r) = kin/h^2 sum_axes sum_{m=-4..4} c_|m| psi(r + m h e_axis)
                + (V(r) + field * x_axis(r)) psi(r)
                + sum_a sum_i p_i^a(r) E_i^a [h^3 sum_{r' in S_a} p_i^a(r') psi(r')]
   for the first nst of ld columns; columns nst..ld-1 of out are untouched.
   Complex-scaled: kin -> kin + i kin_im and V -> V + i V_im. */
void or_hpsi(const or_grid *g, const or_ham *H, double field,
             const cplx *psi, int64_t nst, int64_t ld, cplx *out) {
    const double inv_h2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < g->np; ++p) {
        const int32_t *c = g->ijk + 3 * p;
        double vloc = H->V ? H->V[p] : 0.0;
        if (H->dipole_axis >= 0) vloc += field * coord(g, p, H->dipole_axis);
        const int cs = H->kin_im != 0.0 || H->V_im != NULL;
        const cplx kin_c = H->kin + I * H->kin_im;
        const cplx vloc_c = vloc + I * (H->V_im ? H->V_im[p] : 0.0);
        for (int64_t s = 0; s < nst; ++s) {
            cplx lap = 0.0;
            for (int a = 0; a < 3; ++a) {
                for (int m = -4; m <= 4; ++m) {
                    int32_t q[3] = {c[0], c[1], c[2]};
                    q[a] += m;
                    const int64_t j = lookup(g, q[0], q[1], q[2]);
                    if (j >= 0) lap += FD8[m < 0 ? -m : m] * psi[j * ld + s];
                }
            }
            if (cs)
                out[p * ld + s] = kin_c * inv_h2 * lap + vloc_c * psi[p * ld + s];
            else
                out[p * ld + s] = H->kin * inv_h2 * lap + vloc * psi[p * ld + s];
        }
    }
    /* non-local part, atom by atom in order */
    const double h3 = g->h * g->h * g->h;
    cplx *D = (cplx *)malloc(sizeof(cplx) * 4 * (size_t)(nst > 0 ? nst : 1));
    for (int32_t a = 0; a < H->natoms; ++a) {
        const int64_t e0 = H->kb_off[a], e1 = H->kb_off[a + 1];
        for (int i = 0; i < 4; ++i)
            for (int64_t s = 0; s < nst; ++s) {
                cplx acc = 0.0;
                for (int64_t e = e0; e < e1; ++e)
                    acc += H->kb_p[4 * e + i] * psi[(int64_t)H->kb_idx[e] * ld + s];
                D[i * nst + s] = h3 * acc;
            }
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t r = H->kb_idx[e];
            for (int64_t s = 0; s < nst; ++s) {
                cplx add = 0.0;
                for (int i = 0; i < 4; ++i)
                    add += H->kb_p[4 * e + i] * H->kb_E[4 * a + i] * D[i * nst + s];
                out[r * ld + s] += add;
            }
        }
    }
    free(D);
}

/* ---------------------------------------------------------------------- */
/* Inner products, norms, energy: <a|b> = h^3 sum_r conj(a(r)) b(r).       */
/* ---------------------------------------------------------------------- */

void or_dot(const or_grid *g, const cplx *a, const cplx *b, int64_t nst, int64_t ld, cplx *out) {
    const double h3 = g->h * g->h * g->h;
    for (int64_t s = 0; s < nst; ++s) {
        cplx acc = 0.0;
        for (int64_t p = 0; p < g->np; ++p) acc += conj(a[p * ld + s]) * b[p * ld + s];
        out[s] = h3 * acc;
    }
}

void or_norm2(const or_grid *g, const cplx *a, int64_t nst, int64_t ld, double *out) {
    const double h3 = g->h * g->h * g->h;
    for (int64_t s = 0; s < nst; ++s) {
        double acc = 0.0;
        for (int64_t p = 0; p < g->np; ++p) {
            const cplx v = a[p * ld + s];
            acc += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
        out[s] = h3 * acc;
    }
}

/* Per-orbital <psi_n|H psi_n>; returns the total energy sum_n Re<psi_n|H psi_n>. */
double or_energy(const or_grid *g, const or_ham *H, double field,
                 const cplx *psi, int64_t nst, int64_t ld, cplx *per_orbital) {
    cplx *hp = (cplx *)calloc((size_t)(g->np * ld), sizeof(cplx));
    cplx *d = (cplx *)malloc(sizeof(cplx) * (size_t)(nst > 0 ? nst : 1));
    or_hpsi(g, H, field, psi, nst, ld, hp);
    or_dot(g, psi, hp, nst, ld, d);
    double e = 0.0;
    for (int64_t s = 0; s < nst; ++s) {
        e += creal(d[s]);
        if (per_orbital) per_orbital[s] = d[s];
    }
    free(d);
    free(hp);
    return e;
}

/* ---------------------------------------------------------------------- */
/* Taylor(4) step: psi <- sum_{k=0}^{4} (-i dt H)^k / k! psi, by repeated   */
/* application: t_0 = psi, t_k = (-i dt / k) H t_{k-1}, psi <- sum_k t_k.   */
/* ---------------------------------------------------------------------- */

static void taylor4(const or_grid *g, const or_ham *H, double field, cplx coef_unit,
                    cplx *psi, int64_t nst, int64_t ld) {
    const int64_t n = g->np * ld;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *u = (cplx *)calloc((size_t)n, sizeof(cplx));
    memcpy(t, psi, sizeof(cplx) * (size_t)n);
    for (int k = 1; k <= 4; ++k) {
        or_hpsi(g, H, field, t, nst, ld, u);
        const cplx f = coef_unit / (double)k;
        for (int64_t p = 0; p < g->np; ++p)
            for (int64_t s = 0; s < nst; ++s) {
                t[p * ld + s] = f * u[p * ld + s];
                psi[p * ld + s] += t[p * ld + s];
            }
    }
    free(u);
    free(t);
}

void or_taylor_step(const or_grid *g, const or_ham *H, double dt, double field,
                    cplx *psi, int64_t nst, int64_t ld) {
    taylor4(g, H, field, -I * dt, psi, nst, ld);
}

/* nsteps Taylor(4) steps; step n uses fields[n] (the field at the step
   midpoint), or zero field if fields == NULL. */
void or_propagate(const or_grid *g, const or_ham *H, double dt, int64_t nsteps,
                  const double *fields, cplx *psi, int64_t nst, int64_t ld) {
    for (int64_t n = 0; n < nsteps; ++n)
        taylor4(g, H, fields ? fields[n] : 0.0, -I * dt, psi, nst, ld);
}

/* Mask boundary absorber (section "Photoemission", eq. (mask_split) and the
   outgoing-flow propagation that follows it): after every step the orbital
   keeps only its bounded part, psi <- M(r) U(dt) psi, and the part
   (1 - M) U(dt) psi leaves the simulation box.  removed[s] accumulates, per
   orbital, the charge that leaves the box: the norm before the mask minus
   the norm after it, h^3 sum_r (|U psi|^2 - |M U psi|^2).  M is real. */
void or_propagate_masked(const or_grid *g, const or_ham *H, double dt, int64_t nsteps,
                         const double *fields, const double *mask, cplx *psi, int64_t nst,
                         int64_t ld, double *removed) {
    const double h3 = g->h * g->h * g->h;
    for (int64_t s = 0; s < nst; ++s) removed[s] = 0.0;
    for (int64_t n = 0; n < nsteps; ++n) {
        taylor4(g, H, fields ? fields[n] : 0.0, -I * dt, psi, nst, ld);
        for (int64_t s = 0; s < nst; ++s) {
            double before = 0.0, after = 0.0;
            for (int64_t p = 0; p < g->np; ++p) {
                const cplx u = psi[p * ld + s];
                before += creal(u) * creal(u) + cimag(u) * cimag(u);
                const cplx m = mask[p] * u;
                after += creal(m) * creal(m) + cimag(m) * cimag(m);
                psi[p * ld + s] = m;
            }
            removed[s] += h3 * (before - after);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Optimal control                                                          */
/* ---------------------------------------------------------------------- */

/* E(t) = sum_{k=1}^{K} c_k sin(k pi t / T) */
double or_laser_field(const double *coef, int32_t ncoef, double T, double t) {
    double e = 0.0;
    for (int32_t k = 1; k <= ncoef; ++k) e += coef[k - 1] * sin(k * M_PI * t / T);
    return e;
}

/* Target J = sum_n <psi_n| x_axis |psi_n> (real). */
double or_dipole_target(const or_grid *g, const or_ham *H, const cplx *psi, int64_t nst, int64_t ld) {
    const double h3 = g->h * g->h * g->h;
    double j = 0.0;
    for (int64_t s = 0; s < nst; ++s) {
        double acc = 0.0;
        for (int64_t p = 0; p < g->np; ++p) {
            const cplx v = psi[p * ld + s];
            acc += coord(g, p, H->dipole_axis) * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
        j += h3 * acc;
    }
    return j;
}

/* Forward propagation of nsteps steps under the field built from coef,
   with T = nsteps*dt and step n evaluated at tau_n = (n + 1/2) dt.
   psi is overwritten with psi(T); returns J. */
double or_control_forward(const or_grid *g, const or_ham *H, double dt, int64_t nsteps,
                          const double *coef, int32_t ncoef, cplx *psi, int64_t nst, int64_t ld) {
    const double T = (double)nsteps * dt;
    for (int64_t n = 0; n < nsteps; ++n)
        taylor4(g, H, or_laser_field(coef, ncoef, T, ((double)n + 0.5) * dt), -I * dt, psi, nst, ld);
    return or_dipole_target(g, H, psi, nst, ld);
}

/* One discrete adjoint step for the step psi_{n+1} = T4(-i dt H_n) psi_n.
   Input: psi_n, lambda = lambda_{n+1}.  Output: lambda = T4(-i dt H_n)^dagger
   lambda_{n+1} (= T4(+i dt H_n) lambda_{n+1} since H_n is Hermitian) and
     g_n = dJ/dE_n = 2 Re <lambda_{n+1}| dT4/dE |psi_n>
         = 2 Re sum_{k=1}^{4} a_k sum_{l=0}^{k-1} <H^l lambda| x_axis |H^{k-1-l} psi_n>,
   a_k = (-i dt)^k / k!, grouped by l as sum_l <H^l lambda|x|w_l> with
   w_l = sum_{m=0}^{3-l} a_{l+m+1} H^m psi_n. */
void or_adjoint_step(const or_grid *g, const or_ham *H, double dt, double field,
                     const cplx *psi_n, cplx *lambda, int64_t nst, int64_t ld, double *g_n) {
    const int64_t n = g->np * ld;
    const double h3 = g->h * g->h * g->h;
    cplx *nu[4], *mu[5], *w[4];
    for (int m = 0; m < 4; ++m) nu[m] = (cplx *)calloc((size_t)n, sizeof(cplx));
    for (int l = 0; l < 5; ++l) mu[l] = (cplx *)calloc((size_t)n, sizeof(cplx));
    for (int l = 0; l < 4; ++l) w[l] = (cplx *)calloc((size_t)n, sizeof(cplx));
    memcpy(nu[0], psi_n, sizeof(cplx) * (size_t)n);
    for (int m = 1; m < 4; ++m) or_hpsi(g, H, field, nu[m - 1], nst, ld, nu[m]);
    memcpy(mu[0], lambda, sizeof(cplx) * (size_t)n);
    for (int l = 1; l < 5; ++l) or_hpsi(g, H, field, mu[l - 1], nst, ld, mu[l]);

    cplx a[5];
    a[0] = 1.0;
    for (int k = 1; k < 5; ++k) a[k] = a[k - 1] * (-I * dt) / (double)k;

    for (int l = 0; l < 4; ++l)
        for (int64_t p = 0; p < g->np; ++p)
            for (int64_t s = 0; s < nst; ++s) {
                cplx acc = 0.0;
                for (int m = 0; m <= 3 - l; ++m) acc += a[l + m + 1] * nu[m][p * ld + s];
                w[l][p * ld + s] = acc;
            }

    double gsum = 0.0;
    for (int l = 0; l < 4; ++l)
        for (int64_t s = 0; s < nst; ++s) {
            cplx acc = 0.0;
            for (int64_t p = 0; p < g->np; ++p)
                acc += conj(mu[l][p * ld + s]) * coord(g, p, H->dipole_axis) * w[l][p * ld + s];
            gsum += 2.0 * creal(h3 * acc);
        }
    *g_n = gsum;

    for (int64_t p = 0; p < g->np; ++p)
        for (int64_t s = 0; s < nst; ++s) {
            cplx acc = 0.0;
            for (int k = 0; k < 5; ++k) acc += conj(a[k]) * mu[k][p * ld + s];
            lambda[p * ld + s] = acc;
        }
    for (int m = 0; m < 4; ++m) free(nu[m]);
    for (int l = 0; l < 5; ++l) free(mu[l]);
    for (int l = 0; l < 4; ++l) free(w[l]);
}

/* Gradient of J = sum_n <psi_n(T)|x|psi_n(T)> with respect to the sine
   coefficients: forward pass storing every psi_n, lambda_N = x psi_N,
   backward adjoint steps, dJ/dc_k = sum_n sin(k pi tau_n / T) g_n.
   Writes J, grad[ncoef] and (if non-NULL) g_steps[nsteps]. */
void or_control_gradient(const or_grid *g, const or_ham *H, double dt, int64_t nsteps,
                         const double *coef, int32_t ncoef, const cplx *psi0,
                         int64_t nst, int64_t ld, double *J, double *grad, double *g_steps) {
    const int64_t n = g->np * ld;
    const double T = (double)nsteps * dt;
    cplx *traj = (cplx *)malloc(sizeof(cplx) * (size_t)(n * (nsteps + 1)));
    memcpy(traj, psi0, sizeof(cplx) * (size_t)n);
    for (int64_t k = 0; k < nsteps; ++k) {
        memcpy(traj + (k + 1) * n, traj + k * n, sizeof(cplx) * (size_t)n);
        taylor4(g, H, or_laser_field(coef, ncoef, T, ((double)k + 0.5) * dt), -I * dt,
                traj + (k + 1) * n, nst, ld);
    }
    const cplx *psiN = traj + nsteps * n;
    *J = or_dipole_target(g, H, psiN, nst, ld);

    cplx *lambda = (cplx *)calloc((size_t)n, sizeof(cplx));
    for (int64_t p = 0; p < g->np; ++p)
        for (int64_t s = 0; s < nst; ++s)
            lambda[p * ld + s] = coord(g, p, H->dipole_axis) * psiN[p * ld + s];

    for (int32_t k = 0; k < ncoef; ++k) grad[k] = 0.0;
    for (int64_t step = nsteps - 1; step >= 0; --step) {
        const double tau = ((double)step + 0.5) * dt;
        double gn = 0.0;
        or_adjoint_step(g, H, dt, or_laser_field(coef, ncoef, T, tau), traj + step * n, lambda, nst, ld, &gn);
        if (g_steps) g_steps[step] = gn;
        for (int32_t k = 1; k <= ncoef; ++k) grad[k - 1] += sin(k * M_PI * tau / T) * gn;
    }
    free(lambda);
    free(traj);
}

int32_t or_max_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for the OpenMP loops (timing only; results do not depend on
   it: every output point and every reduction is computed in a fixed order). */
void or_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}
