/* Drives every entry point of the FP64 oracle on small seeded clouds, for a
 * build with the address and undefined-behaviour sanitizers (CPU only). It
 * checks nothing numerically (the pytest pins do that); a sanitizer report
 * or a non-zero exit is the failure. Inputs: a jittered periodic lattice and
 * an open ring of nodes, drawn with a fixed linear congruential generator. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void orc_tables(double *ex, double *ey, double *w, int *opp);
int orc_threads(void);
void orc_set_threads(int t);
void orc_knn(int n, const double *x, const double *y, double Lx, double Ly, int K, int *nbr);
int orc_knn_cand(int n, const double *x, const double *y, double Lx, double Ly, int K, int C,
                 const int *cand, int *nbr);
void orc_owners(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                int mode, int *owner);
int orc_owners_cand(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                    int C, const int *cand, int *owner);
int orc_weights(int n, const double *x, const double *y, double Lx, double Ly, double dx,
                int K, int m, const int *nbr, const int *owner, double *W);
void orc_equilibrium(int n, const double *rho, const double *ux, const double *uy, double *f);
void orc_moments(int n, const double *f, double *rho, double *ux, double *uy);
void orc_run(int n, int K, const int *nbr, const int *owner, const double *W, double tau,
             const double *ax, const double *ay, const unsigned char *node_type, double rho_w,
             int steps, double *f);
void orc_run_links(int n, int K, const int *nbr, const int *owner, const double *W, double tau,
                   const double *ax, const double *ay, const unsigned char *links, int steps,
                   double *f);
void orc_azimuthal_force(int n, const double *x, const double *y, double g,
                         const unsigned char *node_type, double *ax, double *ay);
void orc_lbm_run(int nx, int ny, double tau, int steps, double *f);
void orc_loss_cs(int n, int K, const int *nbr, const int *owner, const double *W,
                 double tau_re, double tau_im, int steps, double rho0, const double *u0x_re,
                 const double *u0x_im, const double *u0y_re, const double *u0y_im,
                 const double *tx, const double *ty, double *J_re, double *J_im);
void orc_adjoint(int n, int K, const int *nbr, const int *owner, const double *W, double tau,
                 int steps, double rho0, const double *u0x, const double *u0y, const double *tx,
                 const double *ty, double *J, double *gx, double *gy, double *gtau);
void orc_stream_transpose(int n, int K, const int *nbr, const int *owner, const double *W,
                          const double *lam, double *out);

static unsigned long long lcg = 12345;
static double uniform(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

static void *must(size_t bytes) {
    void *p = calloc(1, bytes);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* candidate lists by brute force: the C nearest of each query point */
static void candidates(int n, const double *x, const double *y, double L, int nq,
                       const double *qx, const double *qy, int C, int *cand) {
    double *d = must(sizeof(double) * n);
    for (int q = 0; q < nq; ++q) {
        for (int j = 0; j < n; ++j) {
            double dx = x[j] - qx[q], dy = y[j] - qy[q];
            if (L > 0) {
                dx -= L * round(dx / L);
                dy -= L * round(dy / L);
            }
            d[j] = dx * dx + dy * dy;
        }
        for (int c = 0; c < C; ++c) {   /* C passes of selection */
            int best = -1;
            for (int j = 0; j < n; ++j) {
                int taken = 0;
                for (int e = 0; e < c; ++e) taken |= cand[q * C + e] == j;
                if (!taken && (best < 0 || d[j] < d[best])) best = j;
            }
            cand[q * C + c] = best;
        }
    }
    free(d);
}

static void periodic_case(int side, int K, int m, int mode) {
    const int n = side * side;
    const double L = 1.0, h = L / side;
    double *x = must(sizeof(double) * n), *y = must(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        x[i] = fmod((i % side) * h + (uniform() - 0.5) * 0.6 * h + L, L);
        y[i] = fmod((i / side) * h + (uniform() - 0.5) * 0.6 * h + L, L);
    }
    int *nbr = must(sizeof(int) * n * K), *nbr2 = must(sizeof(int) * n * K);
    int *own = must(sizeof(int) * n * 9), *own2 = must(sizeof(int) * n * 9);
    orc_knn(n, x, y, L, L, K, nbr);
    int C = K + 4;
    int *cand = must(sizeof(int) * n * C);
    candidates(n, x, y, L, n, x, y, C, cand);
    orc_knn_cand(n, x, y, L, L, K, C, cand, nbr2);
    orc_owners(n, x, y, L, L, h, mode, own);
    double *px = must(sizeof(double) * n * 8), *py = must(sizeof(double) * n * 8);
    double ex[9], ey[9], w[9];
    int opp[9];
    orc_tables(ex, ey, w, opp);
    for (int i = 0; i < n; ++i)
        for (int k = 1; k < 9; ++k) {
            px[i * 8 + k - 1] = x[i] - ex[k] * h;
            py[i * 8 + k - 1] = y[i] - ey[k] * h;
        }
    int *cand2 = must(sizeof(int) * n * 8 * 2);
    candidates(n, x, y, L, n * 8, px, py, 2, cand2);
    orc_owners_cand(n, x, y, L, L, h, 2, cand2, own2);
    double *W = must(sizeof(double) * n * 9 * K);
    orc_weights(n, x, y, L, L, h, K, m, nbr, own, W);
    double *rho = must(sizeof(double) * n), *ux = must(sizeof(double) * n);
    double *uy = must(sizeof(double) * n), *f = must(sizeof(double) * n * 9);
    for (int i = 0; i < n; ++i) {
        rho[i] = 1.0;
        ux[i] = 0.01 * sin(2 * M_PI * x[i]) * cos(2 * M_PI * y[i]);
        uy[i] = -0.01 * cos(2 * M_PI * x[i]) * sin(2 * M_PI * y[i]);
    }
    orc_equilibrium(n, rho, ux, uy, f);
    orc_run(n, K, nbr, own, W, 0.8, NULL, NULL, NULL, 1.0, 5, f);
    orc_moments(n, f, rho, ux, uy);
    double *zx = must(sizeof(double) * n), *zy = must(sizeof(double) * n);
    double *gx = must(sizeof(double) * n), *gy = must(sizeof(double) * n);
    double J, Ji, gt;
    orc_loss_cs(n, K, nbr, own, W, 0.8, 1e-30, 3, 1.0, ux, zx, uy, zy, zx, zy, &J, &Ji);
    orc_adjoint(n, K, nbr, own, W, 0.8, 3, 1.0, ux, uy, zx, zy, &J, gx, gy, &gt);
    double *lam = must(sizeof(double) * n * 9), *out = must(sizeof(double) * n * 9);
    for (int i = 0; i < n * 9; ++i) lam[i] = uniform();
    orc_stream_transpose(n, K, nbr, own, W, lam, out);
    free(x); free(y); free(nbr); free(nbr2); free(own); free(own2); free(cand); free(cand2);
    free(px); free(py); free(W); free(rho); free(ux); free(uy); free(f); free(zx); free(zy);
    free(gx); free(gy); free(lam); free(out);
}

static void ring_case(void) {
    /* open ring 1 <= r <= 2: wall nodes on both circles, interior at random */
    const int nw = 40, ni = 260, n = 2 * nw + ni, K = 15, m = 2;
    double *x = must(sizeof(double) * n), *y = must(sizeof(double) * n);
    unsigned char *nt = must(n), *links = must(n);
    for (int i = 0; i < nw; ++i) {
        double a = 2 * M_PI * i / nw;
        x[i] = cos(a);
        y[i] = sin(a);
        x[nw + i] = 2 * cos(a);
        y[nw + i] = 2 * sin(a);
        nt[i] = nt[nw + i] = 1;
        links[i] = 0x0f;
        links[nw + i] = 0xf0;
    }
    for (int i = 2 * nw; i < n; ++i) {
        double r = 1.1 + 0.8 * uniform(), a = 2 * M_PI * uniform();
        x[i] = r * cos(a);
        y[i] = r * sin(a);
    }
    int *nbr = must(sizeof(int) * n * K), *own = must(sizeof(int) * n * 9);
    orc_knn(n, x, y, 0.0, 0.0, K, nbr);
    orc_owners(n, x, y, 0.0, 0.0, 0.1, 0, own);
    double *W = must(sizeof(double) * n * 9 * K);
    orc_weights(n, x, y, 0.0, 0.0, 0.1, K, m, nbr, own, W);
    double *ax = must(sizeof(double) * n), *ay = must(sizeof(double) * n);
    orc_azimuthal_force(n, x, y, 1e-5, nt, ax, ay);
    double *rho = must(sizeof(double) * n), *z = must(sizeof(double) * n);
    double *f = must(sizeof(double) * n * 9);
    for (int i = 0; i < n; ++i) rho[i] = 1.0;
    orc_equilibrium(n, rho, z, z, f);
    orc_run(n, K, nbr, own, W, 1.0, ax, ay, nt, 1.0, 5, f);
    orc_run_links(n, K, nbr, own, W, 1.0, ax, ay, links, 5, f);
    free(x); free(y); free(nt); free(links); free(nbr); free(own); free(W); free(ax);
    free(ay); free(rho); free(z); free(f);
}

int main(void) {
    orc_set_threads(2);
    periodic_case(9, 12, 2, 0);
    periodic_case(8, 20, 3, 1);
    periodic_case(11, 30, 4, 0);
    ring_case();
    int nx = 7, ny = 5;
    double *f = must(sizeof(double) * nx * ny * 9);
    for (int i = 0; i < nx * ny * 9; ++i) f[i] = 0.1 + 0.01 * uniform();
    orc_lbm_run(nx, ny, 0.8, 4, f);
    free(f);
    printf("oracle driver done on %d threads\n", orc_threads());
    return 0;
}
