/*
 * lbm_oracle.c -- plain FP64 CPU reference of the D3Q7 multiple-relaxation-time
 * lattice Boltzmann scheme for anisotropic heat conduction (Fang et al.,
 * "Numerical predictions of effective thermal conductivities for 3D
 * four-directional braided composites using the lattice Boltzmann method").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) links, loads or calls this file; only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg do.  It shares no source
 * with the GPU path.
 *
 * The scheme is taken in the paper's own order and notation, without the
 * algebraic shortcuts the GPU path uses:
 *   - equilibrium f_eq (Eq. 6) with gamma = 1/8, epsilon = 2 gamma (Sec. 2.2),
 *   - velocities e_i (Eq. 7), moment matrix M (Eq. 11, c = 1),
 *   - relaxation matrix S as the matrix inverse of the block matrix S^-1 of
 *     Eq. 12 (3x3 tau block, tau_0, tau_4, tau_5, tau_6 on the diagonal),
 *   - tau_ij = delta_ij / 2 + D_ij / epsilon in lattice units (Eq. 13),
 *   - collision f_hat = f - M^-1 S M (f - f_eq)  (Eqs. 5, 8),
 *   - push streaming (Eq. 21) -- unchanged across internal interfaces,
 *     half-way Dirichlet (Eq. 23), Neumann with a given (default zero) flux (Eq. 24)
 *     and periodic (Eq. 25) walls,
 *   - T = sum f (Eq. 14), grad T from the 3x3 system of Eq. 15, heat flux
 *     q = -D grad T (Eq. 16 with the sign of Fourier's law, Eq. 27), and the
 *     effective conductivity of Eq. 22.
 * Lattice units: dx = dt = c = 1.  A phase's lattice diffusivity is
 * D = s k, with one scale s for the whole medium chosen so that the largest
 * eigenvalue of tau - I/2 over all phases equals dmax.
 *
 * The state held between steps is the pre-collision distribution f(x, t).
 * Built with -ffp-contract=off so that no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
static int omp_threads(void) { return omp_get_max_threads(); }
#else
static int omp_threads(void) { return 1; }
#endif

#define Q 7

static const int EV[Q][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5};
static const double GAMMA = 0.125;           /* Sec. 2.2: gamma = 1/8 */
static const double EPS = 2.0 * 0.125;       /* epsilon = 2 gamma     */

enum { SIDE_PERIODIC = 0, SIDE_ADIABATIC = 1, SIDE_DIRICHLET = 2 };

typedef struct {
    int nx, ny, nz;
    long long n;
    int nphase;
    unsigned char *phase;
    double *k;        /* [nphase][9] physical tensors            */
    double *D;        /* [nphase][9] lattice diffusivity s k     */
    double *tau;      /* [nphase][9] tau block of Eq. 12/13      */
    double *omega;    /* [nphase][49] collision matrix of Eq. 8  */
    double s;
    double tau_rest[4]; /* tau_0, tau_4, tau_5, tau_6 */
    int grad_axis;
    double t_hot, t_cold;
    int side[3];
    double qside[3][2];       /* imposed inward heat flux on the two faces of an adiabatic axis (physical) */
    double *f, *fpost, *fnew; /* [Q][n] */
    long long steps;
    double phi_hot, phi_cold; /* wall link fluxes of the last streaming */
    double resid;             /* max |T(t+1) - T(t)| of the last step   */
    int nthreads;
} oracle_ctx;

/* ------------------------------------------------------------------ */
/* small dense linear algebra                                         */
/* ------------------------------------------------------------------ */

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
static int invert(int n, const double *a_in, double *inv) {
    double a[64], b[64];
    memcpy(a, a_in, sizeof(double) * n * n);
    for (int i = 0; i < n * n; i++) b[i] = 0.0;
    for (int i = 0; i < n; i++) b[i * n + i] = 1.0;
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(a[r * n + c]) > fabs(a[piv * n + c])) piv = r;
        if (a[piv * n + c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < n; j++) {
                double t = a[c * n + j]; a[c * n + j] = a[piv * n + j]; a[piv * n + j] = t;
                t = b[c * n + j]; b[c * n + j] = b[piv * n + j]; b[piv * n + j] = t;
            }
        double d = a[c * n + c];
        for (int j = 0; j < n; j++) { a[c * n + j] /= d; b[c * n + j] /= d; }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double m = a[r * n + c];
            if (m == 0.0) continue;
            for (int j = 0; j < n; j++) { a[r * n + j] -= m * a[c * n + j]; b[r * n + j] -= m * b[c * n + j]; }
        }
    }
    memcpy(inv, b, sizeof(double) * n * n);
    return 0;
}

static void matmul(int n, const double *a, const double *b, double *c) {
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double acc = 0.0;
            for (int l = 0; l < n; l++) acc += a[i * n + l] * b[l * n + j];
            c[i * n + j] = acc;
        }
}

/* Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations. */
static void sym3_eigvals(const double *m, double *ev) {
    double a[9];
    memcpy(a, m, sizeof a);
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        if (off < 1e-300) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double apq = a[p * 3 + q];
                if (apq == 0.0) continue;
                double theta = (a[q * 3 + q] - a[p * 3 + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; k++) { /* columns p, q */
                    double akp = a[k * 3 + p], akq = a[k * 3 + q];
                    a[k * 3 + p] = c * akp - s * akq;
                    a[k * 3 + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; k++) { /* rows p, q */
                    double apk = a[p * 3 + k], aqk = a[q * 3 + k];
                    a[p * 3 + k] = c * apk - s * aqk;
                    a[q * 3 + k] = s * apk + c * aqk;
                }
            }
    }
    ev[0] = a[0]; ev[1] = a[4]; ev[2] = a[8];
}

/* 3x3 solve by Gaussian elimination with partial pivoting. */
static void solve3(const double *A, const double *b, double *x) {
    double a[3][4];
    for (int i = 0; i < 3; i++) { for (int j = 0; j < 3; j++) a[i][j] = A[i * 3 + j]; a[i][3] = b[i]; }
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++) if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (piv != c) for (int j = 0; j < 4; j++) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
        for (int r = c + 1; r < 3; r++) {
            double m = a[r][c] / a[c][c];
            for (int j = c; j < 4; j++) a[r][j] -= m * a[c][j];
        }
    }
    for (int i = 2; i >= 0; i--) {
        double acc = a[i][3];
        for (int j = i + 1; j < 3; j++) acc -= a[i][j] * x[j];
        x[i] = acc / a[i][i];
    }
}

/* ------------------------------------------------------------------ */
/* the model of Sec. 2.2                                              */
/* ------------------------------------------------------------------ */

/* Eq. 11 with c = 1: rows are the orthogonal basis vectors phi_k. */
static const double MMAT[Q * Q] = {
    1, 1, 1, 1, 1, 1, 1,
    0, 1, -1, 0, 0, 0, 0,
    0, 0, 0, 1, -1, 0, 0,
    0, 0, 0, 0, 0, 1, -1,
    6, -1, -1, -1, -1, -1, -1,
    0, 2, 2, -1, -1, -1, -1,
    0, 0, 0, 1, 1, -1, -1};

/* Eq. 6 */
static void feq(double T, double *out) {
    out[0] = (1.0 - 6.0 * GAMMA) * T;
    for (int i = 1; i < Q; i++) out[i] = GAMMA * T;
}

/* Build Omega = M^-1 S M for one tau block (Eqs. 8, 12). */
static int build_omega(const double *tau3, const double *tau_rest, double *omega) {
    double sinv[Q * Q] = {0}, S[Q * Q], Minv[Q * Q], tmp[Q * Q];
    sinv[0 * Q + 0] = tau_rest[0];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) sinv[(1 + i) * Q + (1 + j)] = tau3[i * 3 + j];
    sinv[4 * Q + 4] = tau_rest[1];
    sinv[5 * Q + 5] = tau_rest[2];
    sinv[6 * Q + 6] = tau_rest[3];
    if (invert(Q, sinv, S)) return -1;
    if (invert(Q, MMAT, Minv)) return -1;
    matmul(Q, S, MMAT, tmp);
    matmul(Q, Minv, tmp, omega);
    return 0;
}

void oracle_destroy(oracle_ctx *c) {
    if (!c) return;
    free(c->phase); free(c->k); free(c->D); free(c->tau); free(c->omega);
    free(c->f); free(c->fpost); free(c->fnew);
    free(c);
}

/*
 * Create a medium.  k6: [nphase][6] = (kxx, kyy, kzz, kxy, kxz, kyz).
 * tau_rest: (tau_0, tau_4, tau_5, tau_6) or NULL for all ones.
 * Returns NULL when an argument is invalid, a tensor is not symmetric
 * positive definite, or a phase id is out of range.
 */
oracle_ctx *oracle_create(int nx, int ny, int nz, const unsigned char *phase, const double *k6,
                          int nphase, double dmax, const double *tau_rest) {
    if (nx < 1 || ny < 1 || nz < 1 || nphase < 1 || nphase > 256 || !(dmax > 0)) return NULL;
    oracle_ctx *c = (oracle_ctx *)calloc(1, sizeof(oracle_ctx));
    c->nx = nx; c->ny = ny; c->nz = nz; c->n = (long long)nx * ny * nz; c->nphase = nphase;
    c->phase = (unsigned char *)malloc(c->n);
    memcpy(c->phase, phase, c->n);
    for (long long i = 0; i < c->n; i++)
        if (c->phase[i] >= nphase) { oracle_destroy(c); return NULL; }
    c->k = (double *)malloc(sizeof(double) * 9 * nphase);
    c->D = (double *)malloc(sizeof(double) * 9 * nphase);
    c->tau = (double *)malloc(sizeof(double) * 9 * nphase);
    c->omega = (double *)malloc(sizeof(double) * 49 * nphase);
    double lmax = 0.0;
    for (int p = 0; p < nphase; p++) {
        const double *r = k6 + 6 * p;
        double *K = c->k + 9 * p;
        K[0] = r[0]; K[4] = r[1]; K[8] = r[2];
        K[1] = K[3] = r[3]; K[2] = K[6] = r[4]; K[5] = K[7] = r[5];
        double ev[3];
        sym3_eigvals(K, ev);
        for (int i = 0; i < 3; i++) {
            if (!(ev[i] > 0.0)) { oracle_destroy(c); return NULL; }
            if (ev[i] > lmax) lmax = ev[i];
        }
    }
    /* tau - I/2 = D / epsilon = 4 s k; its largest eigenvalue is dmax. */
    c->s = dmax * EPS / lmax;
    for (int i = 0; i < 4; i++) c->tau_rest[i] = tau_rest ? tau_rest[i] : 1.0;
    for (int p = 0; p < nphase; p++) {
        for (int i = 0; i < 9; i++) {
            c->D[9 * p + i] = c->s * c->k[9 * p + i];
            c->tau[9 * p + i] = ((i % 4) == 0 ? 0.5 : 0.0) + c->D[9 * p + i] / EPS; /* Eq. 13 */
        }
        if (build_omega(c->tau + 9 * p, c->tau_rest, c->omega + 49 * p)) { oracle_destroy(c); return NULL; }
    }
    c->f = (double *)calloc(Q * c->n, sizeof(double));
    c->fpost = (double *)calloc(Q * c->n, sizeof(double));
    c->fnew = (double *)calloc(Q * c->n, sizeof(double));
    c->grad_axis = 0; c->t_hot = 1.0; c->t_cold = 0.0;
    c->side[0] = SIDE_DIRICHLET; c->side[1] = SIDE_PERIODIC; c->side[2] = SIDE_PERIODIC;
    c->nthreads = 0;
    return c;
}

double oracle_scale(const oracle_ctx *c) { return c->s; }
void oracle_omega(const oracle_ctx *c, int p, double *out49) { memcpy(out49, c->omega + 49 * p, sizeof(double) * 49); }
void oracle_tau(const oracle_ctx *c, int p, double *out9) { memcpy(out9, c->tau + 9 * p, sizeof(double) * 9); }
long long oracle_steps(const oracle_ctx *c) { return c->steps; }
void oracle_set_threads(oracle_ctx *c, int n) { c->nthreads = n; }

/* grad_axis gets Dirichlet walls: t_hot on its index-0 face, t_cold on its
 * last face.  side[a] for the other axes: 0 periodic, 1 adiabatic. */
int oracle_set_bc(oracle_ctx *c, int grad_axis, double t_hot, double t_cold, const int *side) {
    if (grad_axis < 0 || grad_axis > 2) return -1;
    c->grad_axis = grad_axis; c->t_hot = t_hot; c->t_cold = t_cold;
    memset(c->qside, 0, sizeof(c->qside));
    for (int a = 0; a < 3; a++) {
        if (a == grad_axis) c->side[a] = SIDE_DIRICHLET;
        else {
            if (side[a] != SIDE_PERIODIC && side[a] != SIDE_ADIABATIC) return -1;
            c->side[a] = side[a];
        }
    }
    return 0;
}

/* Neumann faces with a non-zero flux (Eq. 24): q_lo / q_hi = heat flux into
 * the cell through the index-0 / last face of an adiabatic axis, in the
 * units of k times temperature per voxel; the lattice flux phi_n per link
 * and step is s q.  Cleared by oracle_set_bc. */
int oracle_set_side_flux(oracle_ctx *c, int axis, double q_lo, double q_hi) {
    if (axis < 0 || axis > 2 || c->side[axis] != SIDE_ADIABATIC) return -1;
    c->qside[axis][0] = q_lo;
    c->qside[axis][1] = q_hi;
    return 0;
}

/* f(x, 0) = f_eq(T0(x)); T0 = NULL means the zero field. */
void oracle_init(oracle_ctx *c, const double *T0) {
    double e[Q];
    for (long long x = 0; x < c->n; x++) {
        feq(T0 ? T0[x] : 0.0, e);
        for (int i = 0; i < Q; i++) c->f[i * c->n + x] = e[i];
    }
    c->steps = 0; c->phi_hot = c->phi_cold = 0.0; c->resid = 0.0;
}

/*
 * A start that is not at equilibrium: f(x, 0) = f_eq(T0(x)) + e_i . j(x) / 2,
 * the pre-collision flux j read backwards from Eq. 15, j = -epsilon tau grad T0
 * (so that Eq. 15 applied to this state returns grad T0).  The higher moments
 * of Eq. 11 stay at their equilibria.  grad T0 is estimated by central
 * differences over two lattice spacings; at an isothermal wall the wall
 * temperature stands half a spacing beyond the node (the half-way wall of
 * Eq. 23), so that difference spans 1.5 spacings (1 when the axis has a
 * single node); at an adiabatic face the missing neighbour is the node's
 * mirror image, which carries its own value; a periodic axis wraps (Eq. 25).
 */
void oracle_init_flux(oracle_ctx *c, const double *T0) {
    const int dims[3] = {c->nx, c->ny, c->nz};
    const long long stride[3] = {1, c->nx, (long long)c->nx * c->ny};
    for (long long x = 0; x < c->n; x++) {
        const int pos[3] = {(int)(x % c->nx), (int)((x / c->nx) % c->ny), (int)(x / ((long long)c->nx * c->ny))};
        double grad[3];
        for (int a = 0; a < 3; a++) {
            double lo, hi, span = 2.0;
            if (pos[a] > 0) lo = T0[x - stride[a]];
            else if (c->side[a] == SIDE_PERIODIC) lo = T0[x + (long long)(dims[a] - 1) * stride[a]];
            else if (c->side[a] == SIDE_DIRICHLET) { lo = c->t_hot; span -= 0.5; }
            else lo = T0[x];
            if (pos[a] < dims[a] - 1) hi = T0[x + stride[a]];
            else if (c->side[a] == SIDE_PERIODIC) hi = T0[x - (long long)(dims[a] - 1) * stride[a]];
            else if (c->side[a] == SIDE_DIRICHLET) { hi = c->t_cold; span -= 0.5; }
            else hi = T0[x];
            grad[a] = (hi - lo) / span;
        }
        const double *tau = c->tau + 9 * c->phase[x];
        double e[Q];
        feq(T0[x], e);
        for (int i = 0; i < Q; i++) c->f[i * c->n + x] = e[i];
        for (int a = 0; a < 3; a++) {
            const double j = -EPS * (tau[3 * a + 0] * grad[0] + tau[3 * a + 1] * grad[1] + tau[3 * a + 2] * grad[2]);
            c->f[(2 * a + 1) * c->n + x] += 0.5 * j;
            c->f[(2 * a + 2) * c->n + x] -= 0.5 * j;
        }
    }
    c->steps = 0; c->phi_hot = c->phi_cold = 0.0; c->resid = 0.0;
}

/* One node's collision, Eq. 5's right-hand side: f - Omega (f - f_eq). */
void oracle_collide_node(const oracle_ctx *c, int p, const double *fin, double *fout) {
    double T = 0.0, e[Q];
    for (int i = 0; i < Q; i++) T += fin[i];
    feq(T, e);
    const double *om = c->omega + 49 * p;
    for (int i = 0; i < Q; i++) {
        double acc = 0.0;
        for (int j = 0; j < Q; j++) acc += om[i * Q + j] * (fin[j] - e[j]);
        fout[i] = fin[i] - acc;
    }
}

static void one_step(oracle_ctx *c) {
    const long long n = c->n;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int dims[3] = {nx, ny, nz};
    /* collide */
#pragma omp parallel for schedule(static) num_threads(c->nthreads > 0 ? c->nthreads : omp_threads())
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long long idx = ((long long)z * ny + y) * nx + x;
                double fin[Q], fout[Q];
                for (int i = 0; i < Q; i++) fin[i] = c->f[i * n + idx];
                oracle_collide_node(c, c->phase[idx], fin, fout);
                for (int i = 0; i < Q; i++) c->fpost[i * n + idx] = fout[i];
            }
    /* stream (push) with wall treatment */
    double phi_hot = 0.0, phi_cold = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : phi_hot, phi_cold) \
    num_threads(c->nthreads > 0 ? c->nthreads : omp_threads())
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long long idx = ((long long)z * ny + y) * nx + x;
                c->fnew[idx] = c->fpost[idx]; /* rest population stays */
                for (int i = 1; i < Q; i++) {
                    int a = (i - 1) / 2, dir = EV[i][a];
                    int dst[3] = {x + EV[i][0], y + EV[i][1], z + EV[i][2]};
                    int inside = dst[a] >= 0 && dst[a] < dims[a];
                    double fo = c->fpost[i * n + idx];
                    if (inside || c->side[a] == SIDE_PERIODIC) {
                        if (!inside) dst[a] = (dst[a] + dims[a]) % dims[a]; /* Eq. 25 */
                        long long didx = ((long long)dst[2] * ny + dst[1]) * nx + dst[0];
                        c->fnew[i * n + didx] = fo; /* Eq. 21 */
                    } else if (c->side[a] == SIDE_ADIABATIC) {
                        /* Eq. 24 with delta t / delta x = 1: the reflected population
                         * plus the lattice flux entering through this face */
                        c->fnew[OPP[i] * n + idx] = fo + c->s * c->qside[a][dir < 0 ? 0 : 1];
                    } else {
                        double tw = dir < 0 ? c->t_hot : c->t_cold;
                        c->fnew[OPP[i] * n + idx] = -fo + EPS * tw; /* Eq. 23 */
                        if (dir < 0) phi_hot += EPS * tw - 2.0 * fo;
                        else phi_cold += 2.0 * fo - EPS * tw;
                    }
                }
            }
    /* residual: max |T(t+1) - T(t)| */
    double resid = 0.0;
#pragma omp parallel for schedule(static) reduction(max : resid) \
    num_threads(c->nthreads > 0 ? c->nthreads : omp_threads())
    for (long long x = 0; x < n; x++) {
        double t0 = 0.0, t1 = 0.0;
        for (int i = 0; i < Q; i++) { t0 += c->f[i * n + x]; t1 += c->fnew[i * n + x]; }
        double d = fabs(t1 - t0);
        if (d > resid || d != d) resid = d != d ? INFINITY : d;
    }
    double *t = c->f; c->f = c->fnew; c->fnew = t;
    c->phi_hot = phi_hot; c->phi_cold = phi_cold; c->resid = resid;
    c->steps++;
}

void oracle_step(oracle_ctx *c, long long nsteps) {
    for (long long s = 0; s < nsteps; s++) one_step(c);
}

/* T = sum f (Eq. 14). */
void oracle_temperature(const oracle_ctx *c, double *T) {
    for (long long x = 0; x < c->n; x++) {
        double acc = 0.0;
        for (int i = 0; i < Q; i++) acc += c->f[i * c->n + x];
        T[x] = acc;
    }
}

/* grad T from Eq. 15 and q = -D grad T (Eq. 16 with Fourier's sign), both
 * [3][n] in lattice units; either output may be NULL. */
void oracle_flux(const oracle_ctx *c, double *q, double *grad) {
    const long long n = c->n;
    for (long long x = 0; x < n; x++) {
        int p = c->phase[x];
        double rhs[3], g[3];
        for (int a = 0; a < 3; a++) rhs[a] = -(c->f[(2 * a + 1) * n + x] - c->f[(2 * a + 2) * n + x]) / EPS;
        solve3(c->tau + 9 * p, rhs, g);
        const double *D = c->D + 9 * p;
        for (int a = 0; a < 3; a++) {
            if (grad) grad[a * n + x] = g[a];
            if (q) q[a * n + x] = -(D[a * 3 + 0] * g[0] + D[a * 3 + 1] * g[1] + D[a * 3 + 2] * g[2]);
        }
    }
}

/*
 * Effective conductivity (Eq. 22) in physical units, from the current state
 * and the last streaming:
 *   out[0] k_vol   = N_g <q_g> / (dT s)        (volume mean of the node flux)
 *   out[1] k_hot   = N_g Phi_hot / (dT A s)    (hot-wall link flux, A = nodes per face)
 *   out[2] k_cold  = N_g Phi_cold / (dT A s)
 *   out[3..5]      = N_g <q_a> / (dT s), a = x, y, z (column of the tensor)
 *   out[6]         = residual max |dT| of the last step
 */
void oracle_keff(const oracle_ctx *c, double *out) {
    const long long n = c->n;
    double *q = (double *)malloc(sizeof(double) * 3 * n);
    oracle_flux(c, q, NULL);
    int g = c->grad_axis;
    int dims[3] = {c->nx, c->ny, c->nz};
    double ng = dims[g], dT = c->t_hot - c->t_cold, area = (double)n / ng;
    double qm[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++) {
        double acc = 0.0;
        for (long long x = 0; x < n; x++) acc += q[a * n + x];
        qm[a] = acc / (double)n;
    }
    free(q);
    out[0] = ng * qm[g] / (dT * c->s);
    out[1] = ng * c->phi_hot / (dT * area * c->s);
    out[2] = ng * c->phi_cold / (dT * area * c->s);
    for (int a = 0; a < 3; a++) out[3 + a] = ng * qm[a] / (dT * c->s);
    out[6] = c->resid;
}

/*
 * Iterate to steady state.
 *   kind 0: stop when the per-step max |T(t+1) - T(t)| < tol (tested every step).
 *   kind 1: every check_every steps, with k_mid = (k_hot + k_cold) / 2, stop
 *           when |k_hot - k_cold| / k_mid < tol and the relative change of
 *           k_mid since the previous check is < tol / 10.
 * Returns 1 if converged, 0 if max_steps ran out, -1 on a non-finite state.
 * out: as oracle_keff.
 */
int oracle_solve(oracle_ctx *c, double tol, int kind, long long max_steps, int check_every, double *out) {
    double kprev = NAN;
    int conv = 0;
    if (check_every < 1) check_every = 1;
    while (c->steps < max_steps) {
        one_step(c);
        if (!(c->resid < INFINITY)) { oracle_keff(c, out); return -1; }
        if (kind == 0) {
            if (c->resid < tol) { conv = 1; break; }
        } else if (c->steps % check_every == 0) {
            int dims[3] = {c->nx, c->ny, c->nz};
            double ng = dims[c->grad_axis], area = (double)c->n / ng, dT = c->t_hot - c->t_cold;
            double kh = ng * c->phi_hot / (dT * area * c->s), kc = ng * c->phi_cold / (dT * area * c->s);
            double km = 0.5 * (kh + kc);
            /* steady state: what enters through the hot wall and the
             * Neumann faces leaves through the cold wall */
            double side_in = 0.0;
            for (int a = 0; a < 3; a++)
                side_in += c->s * (c->qside[a][0] + c->qside[a][1]) * ((double)c->n / dims[a]);
            double ks = ng * side_in / (dT * area * c->s);
            int gap_ok = fabs(kh - kc + ks) < tol * fabs(km);
            int chg_ok = kprev == kprev && fabs(km - kprev) < 0.1 * tol * fabs(km);
            kprev = km;
            if (gap_ok && chg_ok) { conv = 1; break; }
        }
    }
    oracle_keff(c, out);
    return conv;
}

void oracle_get_f(const oracle_ctx *c, double *f) { memcpy(f, c->f, sizeof(double) * Q * c->n); }
void oracle_set_f(oracle_ctx *c, const double *f) { memcpy(c->f, f, sizeof(double) * Q * c->n); }
void oracle_last_fluxes(const oracle_ctx *c, double *out3) {
    out3[0] = c->phi_hot; out3[1] = c->phi_cold; out3[2] = c->resid;
}
