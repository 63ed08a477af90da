/* Plain FP64 CPU oracle of the Meshless Lattice Boltzmann Method (MLBM).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference that the GPU library is
 * checked against; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code, header, table or helper with
 * the GPU library and must never be linked into it.
 *
 * It follows the paper (Strzelczyk & Matyka, "Study of the convergence of the
 * Meshless Lattice Boltzmann Method in Taylor-Green and annular channel
 * flows") step by step, in its notation where possible:
 *   - D2Q9 velocities and weights, equilibrium, BGK collision, moments:
 *     Sec. 2.1 (eqs. LBM_streaming, LBM_collision, feq, macro_var);
 *   - RBF interpolation with polynomial augmentation, shape vectors:
 *     Sec. 2.2 (eqs. rbf_interp_set_augmented, shape_vector, poly_sets),
 *     solved by LU with partial pivoting (Sec. 2.3);
 *   - the semi-Lagrangian MLBM loop: Sec. 2.3 and Appendix A (Algorithm 1);
 *   - body force and walls of the annulus: Sec. 3.
 * Everything is double precision. Layouts are node-major:
 *   nbr [n][K], owner [n][9], W [n][9][K], f [n][9].
 * Loops over nodes are parallelised with OpenMP; results do not depend on the
 * thread count (no cross-thread reductions in floating point).
 *
 * Build with -ffp-contract=off so that squared distances are rounded exactly as
 * written (kNN ties are broken on bitwise equal distances, then by index).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* D2Q9 directions in the order of Sec. 2.1 and their weights w_k. */
static const double EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const double EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double OMEGA[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

#define SCALAR double
#define FN(name) name##_r
#include "lbm_core.inc"
#undef SCALAR
#undef FN

#define SCALAR double complex
#define FN(name) name##_c
#include "lbm_core.inc"
#undef SCALAR
#undef FN

/* ------------------------------------------------------------------------ */
/* Tables and thread count                                                  */
/* ------------------------------------------------------------------------ */

void orc_tables(double *ex, double *ey, double *w, int *opp) {
    for (int k = 0; k < Q; ++k) {
        ex[k] = EX[k];
        ey[k] = EY[k];
        w[k] = OMEGA[k];
        opp[k] = OPP[k];
    }
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel loops (results do not depend on it). */
void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Geometry: periodic minimum image, stencils, closest Eulerian node         */
/* ------------------------------------------------------------------------ */

/* Shortest signed separation along one axis of period L (L <= 0: open). */
static double min_image(double d, double L) {
    if (L > 0.0) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

static double dist2(double ax, double ay, double bx, double by, double Lx, double Ly) {
    double dx = min_image(bx - ax, Lx);
    double dy = min_image(by - ay, Ly);
    return dx * dx + dy * dy;
}

/* Stencil X^L of node c (Sec. 2.2): c itself first, then its K-1 closest other
 * nodes by (squared distance, index), searched over all nodes (brute force).
 * Periodicity is the minimum image (Sec. 3: periodic search of stencil members). */
void orc_knn_one(int n, const double *x, const double *y, double Lx, double Ly, int K,
                 int c, int *out) {
    double bd[K];
    int bj[K];
    int have = 0; /* filled entries among positions 1..K-1 */
    out[0] = c;
    for (int j = 0; j < n; ++j) {
        if (j == c) continue;
        double d = dist2(x[c], y[c], x[j], y[j], Lx, Ly);
        /* insertion into the sorted list bd[1..have] */
        if (have == K - 1) {
            if (d > bd[K - 1] || (d == bd[K - 1] && j > bj[K - 1])) continue;
            have--; /* drop the last */
        }
        int pos = have + 1;
        while (pos > 1 && (bd[pos - 1] > d || (bd[pos - 1] == d && bj[pos - 1] > j))) {
            bd[pos] = bd[pos - 1];
            bj[pos] = bj[pos - 1];
            pos--;
        }
        bd[pos] = d;
        bj[pos] = j;
        have++;
    }
    for (int q = 1; q < K; ++q) out[q] = (q <= have) ? bj[q] : -1;
}

void orc_knn(int n, const double *x, const double *y, double Lx, double Ly, int K,
             int *nbr) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) orc_knn_one(n, x, y, Lx, Ly, K, i, nbr + (size_t)i * K);
}

/* Closest Eulerian node to the point (px, py); ties go to the lower index. */
int orc_nearest(int n, const double *x, const double *y, double Lx, double Ly, double px,
                double py) {
    int best = -1;
    double bd = INFINITY;
    for (int j = 0; j < n; ++j) {
        double d = dist2(px, py, x[j], y[j], Lx, Ly);
        if (d < bd) {
            bd = d;
            best = j;
        }
    }
    return best;
}

/* Owner of each Lagrangian (departure) point (Sec. 2.3, Appendix A): the
 * population k arriving at x_i departs from p = x_i - e_k dx. In mode 0 (the
 * paper's text) the owner is the closest Eulerian node to p; in mode 1 every
 * departure point of node i uses node i's own stencil. k = 0 departs from x_i
 * itself, whose closest node is i. owner: [n][9]. */
void orc_owners(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                int mode, int *owner) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        owner[(size_t)i * Q] = i;
        for (int k = 1; k < Q; ++k) {
            if (mode == 1) {
                owner[(size_t)i * Q + k] = i;
            } else {
                double px = x[i] - EX[k] * dx, py = y[i] - EY[k] * dx;
                owner[(size_t)i * Q + k] = orc_nearest(n, x, y, Lx, Ly, px, py);
            }
        }
    }
}

/* The same two searches for large clouds, from candidate lists that a spatial
 * search library (a k-d tree) produced: cand[q][0..C-1] are C distinct nodes
 * that it reports as the C nearest to query point q. The answer is taken from
 * the candidates by the exact rule above (squared distance as written here,
 * then index). It is provably the brute-force answer when every chosen
 * distance is clearly below the farthest candidate's, since no node outside
 * the list is nearer than that one (the margin 1e-9 covers the library's own
 * rounding); otherwise that query falls back to the brute-force search. Each
 * function returns how many queries fell back. */
static const double CAND_MARGIN = 1.0 - 1e-9;

int orc_knn_cand(int n, const double *x, const double *y, double Lx, double Ly, int K, int C,
                 const int *cand, int *nbr) {
    int fallbacks = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : fallbacks)
    for (int c = 0; c < n; ++c) {
        const int *cq = cand + (size_t)c * C;
        double bd[K];
        int bj[K];
        int have = 0, self = 0;
        double dmax = 0.0;
        int *out = nbr + (size_t)c * K;
        out[0] = c;
        for (int e = 0; e < C; ++e) {
            int j = cq[e];
            double d = dist2(x[c], y[c], x[j], y[j], Lx, Ly);
            if (d > dmax) dmax = d;
            if (j == c) {
                self = 1;
                continue;
            }
            if (have == K - 1) {
                if (d > bd[K - 1] || (d == bd[K - 1] && j > bj[K - 1])) continue;
                have--;
            }
            int pos = have + 1;
            while (pos > 1 && (bd[pos - 1] > d || (bd[pos - 1] == d && bj[pos - 1] > j))) {
                bd[pos] = bd[pos - 1];
                bj[pos] = bj[pos - 1];
                pos--;
            }
            bd[pos] = d;
            bj[pos] = j;
            have++;
        }
        if (self && have == K - 1 && bd[K - 1] < dmax * CAND_MARGIN) {
            for (int q = 1; q < K; ++q) out[q] = bj[q];
        } else {
            orc_knn_one(n, x, y, Lx, Ly, K, c, out);
            fallbacks++;
        }
    }
    return fallbacks;
}

/* Owners of the departure points (mode 0 of orc_owners) from candidate lists
 * of the points x_i - e_k dx, k = 1..8: cand[(i * 8 + k - 1)][0..C-1]. */
int orc_owners_cand(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                    int C, const int *cand, int *owner) {
    int fallbacks = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : fallbacks)
    for (int i = 0; i < n; ++i) {
        owner[(size_t)i * Q] = i;
        for (int k = 1; k < Q; ++k) {
            double px = x[i] - EX[k] * dx, py = y[i] - EY[k] * dx;
            const int *cq = cand + ((size_t)i * 8 + (k - 1)) * C;
            int best = -1;
            double bd = INFINITY, dmax = 0.0;
            for (int e = 0; e < C; ++e) {
                int j = cq[e];
                double d = dist2(px, py, x[j], y[j], Lx, Ly);
                if (d > dmax) dmax = d;
                if (d < bd || (d == bd && j < best)) {
                    bd = d;
                    best = j;
                }
            }
            if (!(best >= 0 && bd < dmax * CAND_MARGIN)) {
                best = orc_nearest(n, x, y, Lx, Ly, px, py);
                fallbacks++;
            }
            owner[(size_t)i * Q + k] = best;
        }
    }
    return fallbacks;
}

/* ------------------------------------------------------------------------ */
/* RBF interpolation with polynomial augmentation                           */
/* ------------------------------------------------------------------------ */

/* Number of 2-D monomials of total degree <= m. */
int orc_poly_count(int m) { return (m + 1) * (m + 2) / 2; }

/* Monomials in the order of eq. poly_sets: 1, x, y, x^2, xy, y^2, x^3, x^2y,
 * xy^2, y^3, x^4, x^3y, x^2y^2, xy^3, y^4 (truncated at degree m). */
static void monomials(int m, double px, double py, double *out) {
    int q = 0;
    for (int deg = 0; deg <= m; ++deg)
        for (int a = 0; a <= deg; ++a) out[q++] = pow(px, deg - a) * pow(py, a);
}

/* Local collocation system of eq. rbf_interp_set_augmented and the right-hand
 * side of eq. shape_vector for the point p. The stencil coordinates (rx, ry)
 * and p are given relative to the stencil centre; they are divided by the
 * stencil radius max_j |r_j| (the interpolant of r^3 plus complete polynomials
 * is invariant under this scaling; it only improves conditioning).
 * Phi: [(K+M)][(K+M)] row-major, phi: [K+M]. Returns K+M. */
int orc_local_system(int K, int m, const double *rx, const double *ry, double px,
                     double py, double *Phi, double *phi) {
    int M = orc_poly_count(m), nn = K + M;
    double rad = 0.0;
    for (int j = 0; j < K; ++j) {
        double r = sqrt(rx[j] * rx[j] + ry[j] * ry[j]);
        if (r > rad) rad = r;
    }
    if (rad <= 0.0) rad = 1.0;
    double sx[K], sy[K], mono[M];
    for (int j = 0; j < K; ++j) {
        sx[j] = rx[j] / rad;
        sy[j] = ry[j] / rad;
    }
    double qx = px / rad, qy = py / rad;
    for (int a = 0; a < nn * nn; ++a) Phi[a] = 0.0;
    for (int a = 0; a < K; ++a) {
        for (int b = 0; b < K; ++b) {
            double dx = sx[a] - sx[b], dy = sy[a] - sy[b];
            double r = sqrt(dx * dx + dy * dy);
            Phi[a * nn + b] = r * r * r; /* R_L: phi(r) = r^3 */
        }
        monomials(m, sx[a], sy[a], mono);
        for (int q = 0; q < M; ++q) {
            Phi[a * nn + K + q] = mono[q];   /* P_L   */
            Phi[(K + q) * nn + a] = mono[q]; /* P_L^T */
        }
    }
    for (int j = 0; j < K; ++j) {
        double dx = sx[j] - qx, dy = sy[j] - qy;
        double r = sqrt(dx * dx + dy * dy);
        phi[j] = r * r * r;
    }
    monomials(m, qx, qy, mono);
    for (int q = 0; q < M; ++q) phi[K + q] = mono[q];
    return nn;
}

/* Solve A x = b by LU decomposition with partial pivoting (row interchanges,
 * Doolittle form, unit lower factor). A is overwritten by its factors. Returns
 * 0, or 1 if a pivot is below 1e3 * eps * ||A||_inf (numerically singular). */
int orc_lu_solve(int nn, double *A, const double *b, double *xout) {
    int perm[nn];
    double norm = 0.0;
    for (int r = 0; r < nn; ++r) {
        double s = 0.0;
        for (int c = 0; c < nn; ++c) s += fabs(A[r * nn + c]);
        if (s > norm) norm = s;
        perm[r] = r;
    }
    double tiny = 1e3 * 2.220446049250313e-16 * norm;
    for (int k = 0; k < nn; ++k) {
        int p = k;
        for (int r = k + 1; r < nn; ++r)
            if (fabs(A[r * nn + k]) > fabs(A[p * nn + k])) p = r;
        if (!(fabs(A[p * nn + k]) > tiny)) return 1;
        if (p != k) {
            for (int c = 0; c < nn; ++c) {
                double t = A[k * nn + c];
                A[k * nn + c] = A[p * nn + c];
                A[p * nn + c] = t;
            }
            int t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
        for (int r = k + 1; r < nn; ++r) {
            double l = A[r * nn + k] / A[k * nn + k];
            A[r * nn + k] = l;
            for (int c = k + 1; c < nn; ++c) A[r * nn + c] -= l * A[k * nn + c];
        }
    }
    double yv[nn];
    for (int r = 0; r < nn; ++r) { /* L y = P b */
        double s = b[perm[r]];
        for (int c = 0; c < r; ++c) s -= A[r * nn + c] * yv[c];
        yv[r] = s;
    }
    for (int r = nn - 1; r >= 0; --r) { /* U x = y */
        double s = yv[r];
        for (int c = r + 1; c < nn; ++c) s -= A[r * nn + c] * xout[c];
        xout[r] = s / A[r * nn + r];
    }
    return 0;
}

/* Shape vector w_L(p) of eq. shape_vector: the first K entries of
 * Phi^{-1} phi_L(p). Phi is symmetric, so this is also the vector that dots
 * the data f_L with the interpolant's value. Returns 0 or 1 (singular). */
int orc_shape_vector(int K, int m, const double *rx, const double *ry, double px,
                     double py, double *w) {
    int nn = K + orc_poly_count(m);
    double *Phi = malloc(sizeof(double) * nn * nn);
    double phi[nn], sol[nn];
    orc_local_system(K, m, rx, ry, px, py, Phi, phi);
    int st = orc_lu_solve(nn, Phi, phi, sol);
    free(Phi);
    for (int j = 0; j < K; ++j) w[j] = sol[j];
    return st;
}

/* Shape vectors of every departure point (Appendix A, initialisation loop):
 * for node i and direction k, stencil of the owner s, coordinates taken
 * relative to x_s through the minimum image. W: [n][9][K].
 * Returns 0, or -(1 + i) for the first node i whose local system is singular. */
int orc_weights(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                int K, int m, const int *nbr, const int *owner, double *W) {
    int bad = n;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : bad)
    for (int i = 0; i < n; ++i) {
        double rx[K], ry[K];
        for (int k = 0; k < Q; ++k) {
            int s = owner[(size_t)i * Q + k];
            const int *st = nbr + (size_t)s * K;
            for (int j = 0; j < K; ++j) {
                rx[j] = min_image(x[st[j]] - x[s], Lx);
                ry[j] = min_image(y[st[j]] - y[s], Ly);
            }
            double px = min_image(x[i] - EX[k] * dx - x[s], Lx);
            double py = min_image(y[i] - EY[k] * dx - y[s], Ly);
            if (orc_shape_vector(K, m, rx, ry, px, py, W + ((size_t)i * Q + k) * K))
                if (i < bad) bad = i;
        }
    }
    return bad < n ? -(1 + bad) : 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice Boltzmann pieces (real scalar)                                    */
/* ------------------------------------------------------------------------ */

void orc_feq(double rho, double ux, double uy, double *out) { feq_r(rho, ux, uy, out); }

void orc_equilibrium(int n, const double *rho, const double *ux, const double *uy,
                     double *f) {
    for (int i = 0; i < n; ++i) feq_r(rho[i], ux[i], uy[i], f + (size_t)i * Q);
}

void orc_moments(int n, const double *f, double *rho, double *ux, double *uy) {
    for (int i = 0; i < n; ++i) moments1_r(f + (size_t)i * Q, rho + i, ux + i, uy + i);
}

void orc_collide(int n, const double *f, double tau, const double *ax, const double *ay,
                 const unsigned char *node_type, double *fpost) {
    collide_all_r(n, f, tau, ax, ay, node_type, fpost);
}

void orc_stream(int n, int K, const int *nbr, const int *owner, const double *W,
                const double *fpost, double *f) {
    stream_all_r(n, K, nbr, owner, W, fpost, f);
}

void orc_walls(int n, const unsigned char *node_type, double rho_w, double *f) {
    walls_r(n, node_type, rho_w, f);
}

/* Constant acceleration g along the azimuthal direction about the origin
 * (Sec. 3): a(x) = g (-y, x) / r at fluid nodes, zero at wall nodes. */
void orc_azimuthal_force(int n, const double *x, const double *y, double g,
                         const unsigned char *node_type, double *ax, double *ay) {
    for (int i = 0; i < n; ++i) {
        double r = sqrt(x[i] * x[i] + y[i] * y[i]);
        int wall = node_type && node_type[i];
        ax[i] = (wall || r == 0.0) ? 0.0 : -g * y[i] / r;
        ay[i] = (wall || r == 0.0) ? 0.0 : g * x[i] / r;
    }
}

/* Run `steps` timesteps from the populations f (in place). */
void orc_run(int n, int K, const int *nbr, const int *owner, const double *W, double tau,
             const double *ax, const double *ay, const unsigned char *node_type,
             double rho_w, int steps, double *f) {
    double *tmp = malloc(sizeof(double) * (size_t)n * Q);
    for (int t = 0; t < steps; ++t)
        step_r(n, K, nbr, owner, W, tau, ax, ay, node_type, rho_w, f, tmp);
    free(tmp);
}

/* Bounce-back walls (Sec. 3, annular channel): per step COLLIDE with the
 * body force at every node, STREAM, then the reflection of the flagged
 * populations at wall nodes (links: [n], bit k-1 = direction k enters from
 * outside). f: [n][9], updated in place. */
void orc_run_links(int n, int K, const int *nbr, const int *owner, const double *W, double tau,
                   const double *ax, const double *ay, const unsigned char *links, int steps,
                   double *f) {
    double *tmp = malloc(sizeof(double) * (size_t)n * Q);
    for (int t = 0; t < steps; ++t) {
        collide_all_r(n, f, tau, ax, ay, NULL, tmp);
        stream_all_r(n, K, nbr, owner, W, tmp, f);
        bounce_r(n, links, f);
    }
    free(tmp);
}

void orc_bounce(int n, const unsigned char *links, double *f) { bounce_r(n, links, f); }

/* Standard LBM on a periodic nx x ny lattice (node index iy*nx + ix): BGK
 * collision then index-shift streaming f_k(x) = f_k^post(x - e_k)
 * (eq. LBM_streaming). f: [nx*ny][9], updated in place. */
void orc_lbm_run(int nx, int ny, double tau, int steps, double *f) {
    int n = nx * ny;
    double *post = malloc(sizeof(double) * (size_t)n * Q);
    for (int t = 0; t < steps; ++t) {
        collide_all_r(n, f, tau, NULL, NULL, NULL, post);
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix)
                for (int k = 0; k < Q; ++k) {
                    int sx = ((ix - (int)EX[k]) % nx + nx) % nx;
                    int sy = ((iy - (int)EY[k]) % ny + ny) % ny;
                    f[((size_t)iy * nx + ix) * Q + k] = post[((size_t)sy * nx + sx) * Q + k];
                }
    }
    free(post);
}

/* ------------------------------------------------------------------------ */
/* Differentiation of a periodic rollout (no walls, no force)                */
/* ------------------------------------------------------------------------ */

/* Loss after `steps` steps from f0 = feq(rho0, u0):
 * J = 1/2 sum_i |u_i(f^T) - u*_i|^2. Complex-step variant: u0 and tau carry
 * imaginary parts (perturbation directions times the step), and the imaginary
 * part of J is returned as well. */
void orc_loss_cs(int n, int K, const int *nbr, const int *owner, const double *W,
                 double tau_re, double tau_im, int steps, double rho0,
                 const double *u0x_re, const double *u0x_im, const double *u0y_re,
                 const double *u0y_im, const double *tx, const double *ty,
                 double *J_re, double *J_im) {
    double complex *f = malloc(sizeof(double complex) * (size_t)n * Q);
    double complex *tmp = malloc(sizeof(double complex) * (size_t)n * Q);
    double complex tau = tau_re + I * tau_im;
    for (int i = 0; i < n; ++i)
        feq_c(rho0, u0x_re[i] + I * u0x_im[i], u0y_re[i] + I * u0y_im[i],
              f + (size_t)i * Q);
    for (int t = 0; t < steps; ++t)
        step_c(n, K, nbr, owner, W, tau, NULL, NULL, NULL, 0.0, f, tmp);
    double complex J = velocity_misfit_c(n, f, tx, ty);
    *J_re = creal(J);
    *J_im = cimag(J);
    free(f);
    free(tmp);
}

/* Jacobian of the BGK collision at one node, C[a][b] = d fpost_a / d f_b,
 * from the chain rule through rho = sum f and j = sum f e (no force):
 *   d feq_a / d rho = w_a [1 - (e_a.u)^2 / (2 cs^4) + u^2 / (2 cs^2)],
 *   d feq_a / d j   = w_a [e_a / cs^2 + (e_a.u) e_a / cs^4 - u / cs^2]. */
static void collision_jacobian(const double *f, double tau, double C[Q][Q]) {
    const double cs2 = 1.0 / 3.0;
    double rho, ux, uy;
    moments1_r(f, &rho, &ux, &uy);
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < Q; ++a) {
        double cu = EX[a] * ux + EY[a] * uy;
        double drho = OMEGA[a] * (1.0 - cu * cu / (2 * cs2 * cs2) + uu / (2 * cs2));
        double djx = OMEGA[a] * (EX[a] / cs2 + cu * EX[a] / (cs2 * cs2) - ux / cs2);
        double djy = OMEGA[a] * (EY[a] / cs2 + cu * EY[a] / (cs2 * cs2) - uy / cs2);
        for (int b = 0; b < Q; ++b) {
            double dfeq = drho + djx * EX[b] + djy * EY[b];
            C[a][b] = (a == b ? 1.0 - 1.0 / tau : 0.0) + dfeq / tau;
        }
    }
}

/* Reverse-mode gradient of J with respect to u0 ([n] each) and tau by the
 * discrete adjoint of the rollout: forward states f^0..f^T are stored, the
 * adjoint of f^T is dJ/df^T, and for each step in reverse the adjoint of the
 * post-collision state is the transpose of streaming (a scatter over the same
 * weights), and the adjoint of f^n is the transposed collision Jacobian
 * applied to it. dJ/dtau collects lam_post . d fpost / d tau at every step;
 * dJ/du0 is the transpose of d feq / d u at t = 0 applied to lam f^0. */
void orc_adjoint(int n, int K, const int *nbr, const int *owner, const double *W,
                 double tau, int steps, double rho0, const double *u0x, const double *u0y,
                 const double *tx, const double *ty, double *J, double *gx, double *gy,
                 double *gtau) {
    size_t nq = (size_t)n * Q;
    double *fs = malloc(sizeof(double) * nq * (size_t)(steps + 1));
    double *tmp = malloc(sizeof(double) * nq);
    double *lam = malloc(sizeof(double) * nq);
    double *lamp = malloc(sizeof(double) * nq);
    for (int i = 0; i < n; ++i) feq_r(rho0, u0x[i], u0y[i], fs + (size_t)i * Q);
    for (int t = 0; t < steps; ++t) {
        memcpy(fs + nq * (t + 1), fs + nq * t, sizeof(double) * nq);
        step_r(n, K, nbr, owner, W, tau, NULL, NULL, NULL, 0.0, fs + nq * (t + 1), tmp);
    }
    const double *fT = fs + nq * steps;
    *J = velocity_misfit_r(n, fT, tx, ty);
    /* dJ/df_b = sum_c (u_c - u*_c) (e_bc - u_c) / rho */
    for (int i = 0; i < n; ++i) {
        double rho, ux, uy;
        moments1_r(fT + (size_t)i * Q, &rho, &ux, &uy);
        double rx = ux - tx[i], ry = uy - ty[i];
        for (int b = 0; b < Q; ++b)
            lam[(size_t)i * Q + b] = (rx * (EX[b] - ux) + ry * (EY[b] - uy)) / rho;
    }
    double dtau = 0.0;
    for (int t = steps - 1; t >= 0; --t) {
        const double *fn = fs + nq * t;
        /* transpose of streaming: scatter-add */
        memset(lamp, 0, sizeof(double) * nq);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < Q; ++k) {
                int s = owner[(size_t)i * Q + k];
                const double *w = W + ((size_t)i * Q + k) * K;
                for (int j = 0; j < K; ++j)
                    lamp[(size_t)nbr[(size_t)s * K + j] * Q + k] += w[j] * lam[(size_t)i * Q + k];
            }
        /* transpose of collision, and d fpost / d tau = (f - feq) / tau^2 */
        for (int i = 0; i < n; ++i) {
            double C[Q][Q], eq[Q], rho, ux, uy;
            const double *fi = fn + (size_t)i * Q;
            collision_jacobian(fi, tau, C);
            moments1_r(fi, &rho, &ux, &uy);
            feq_r(rho, ux, uy, eq);
            for (int b = 0; b < Q; ++b) {
                double s = 0.0;
                for (int a = 0; a < Q; ++a) s += C[a][b] * lamp[(size_t)i * Q + a];
                lam[(size_t)i * Q + b] = s;
            }
            for (int a = 0; a < Q; ++a)
                dtau += lamp[(size_t)i * Q + a] * (fi[a] - eq[a]) / (tau * tau);
        }
    }
    /* d feq_k / d u at rho0, u0 */
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < n; ++i) {
        double ux = u0x[i], uy = u0y[i], sx = 0.0, sy = 0.0;
        for (int k = 0; k < Q; ++k) {
            double cu = EX[k] * ux + EY[k] * uy;
            double l = lam[(size_t)i * Q + k];
            sx += l * OMEGA[k] * rho0 * (EX[k] / cs2 + cu * EX[k] / (cs2 * cs2) - ux / cs2);
            sy += l * OMEGA[k] * rho0 * (EY[k] / cs2 + cu * EY[k] / (cs2 * cs2) - uy / cs2);
        }
        gx[i] = sx;
        gy[i] = sy;
    }
    *gtau = dtau;
    free(fs);
    free(tmp);
    free(lam);
    free(lamp);
}

/* Transpose of streaming alone, for dot-product tests: out = S^T lam. */
void orc_stream_transpose(int n, int K, const int *nbr, const int *owner, const double *W,
                          const double *lam, double *out) {
    memset(out, 0, sizeof(double) * (size_t)n * Q);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < Q; ++k) {
            int s = owner[(size_t)i * Q + k];
            const double *w = W + ((size_t)i * Q + k) * K;
            for (int j = 0; j < K; ++j)
                out[(size_t)nbr[(size_t)s * K + j] * Q + k] += w[j] * lam[(size_t)i * Q + k];
        }
}
