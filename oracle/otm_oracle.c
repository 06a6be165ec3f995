/*
 * Plain FP64 CPU oracle for the periodic thermal homogenization step
 * (Quan, Zhai, Fu: "OpenTM", arXiv 2405.19991).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests and the CPU baseline can check the
 * HIP path against an obviously correct, slow implementation written straight
 * from the paper's definitions:
 *
 *   - unit-voxel trilinear hex conduction matrix, by Gauss quadrature
 *     (FE equilibrium K T = f, Sec. 2.1);
 *   - assembled periodic stiffness in CSR, A = sum_e k_e P_e^T Khat P_e, and
 *     the three macro loads b^i = sum_e k_e P_e^T Khat X_i
 *     (periodic BCs and the three test gradients, Sec. 2.2);
 *   - unpreconditioned conjugate gradients on the zero-mean subspace;
 *   - homogenized tensor kappa_ij = N^-3 sum_e k_e (X_i - chi^i_e)^T Khat
 *     (X_j - chi^j_e) (discrete homogenization formula, Sec. 2.2);
 *   - SIMP k_e = kmin + rho~_e^p (k0 - kmin) (Sec. 2.2);
 *   - density filter as a normalized weighted average (Sec. 2.3) with a
 *     separable periodic hat weight, and its transpose;
 *   - element sensitivities d kappa_ij / d rho~_e (Sec. 2.3, sensitivity
 *     equation, with the factor (k0 - kmin) of the SIMP derivative);
 *   - Optimality Criteria update by bisection on the multiplier.
 *
 * Grid convention: N^3 elements and N^3 nodes on a periodic cell; node
 * (i,j,k) is the lower corner of element (i,j,k); flat index i + N*(j+N*k).
 * Local vertex l of an element has offset (l&1, (l>>1)&1, (l>>2)&1).
 * Everything is float64 and written for clarity, not speed; OpenMP only
 * parallelizes independent loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t wrap(int64_t a, int64_t n) {
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

static int64_t node_index(int64_t i, int64_t j, int64_t k, int64_t n) {
    return wrap(i, n) + n * (wrap(j, n) + n * wrap(k, n));
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Element matrix: K_lm = integral over [0,1]^3 of grad N_l . grad N_m with   */
/* trilinear N_l(x) = prod_a phi_{l_a}(x_a), phi_0 = 1-t, phi_1 = t.  The      */
/* integrand is at most quadratic per coordinate, so 2-point Gauss-Legendre   */
/* per axis is exact.                                                          */
/* ------------------------------------------------------------------------ */
static double phi(int bit, double t) { return bit ? t : 1.0 - t; }
static double dphi(int bit) { return bit ? 1.0 : -1.0; }

void ora_element_matrix(double *K /* 64, row-major [l][m] */) {
    const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const double w = 0.125; /* (1/2)^3: Gauss weights on [0,1] */
    memset(K, 0, 64 * sizeof(double));
    for (int qa = 0; qa < 2; ++qa)
        for (int qb = 0; qb < 2; ++qb)
            for (int qc = 0; qc < 2; ++qc) {
                double x[3] = {g[qa], g[qb], g[qc]};
                double grad[8][3];
                for (int l = 0; l < 8; ++l) {
                    int bits[3] = {l & 1, (l >> 1) & 1, (l >> 2) & 1};
                    for (int a = 0; a < 3; ++a) {
                        double v = dphi(bits[a]);
                        for (int b2 = 0; b2 < 3; ++b2)
                            if (b2 != a) v *= phi(bits[b2], x[b2]);
                        grad[l][a] = v;
                    }
                }
                for (int l = 0; l < 8; ++l)
                    for (int m = 0; m < 8; ++m)
                        K[l * 8 + m] += w * (grad[l][0] * grad[m][0] + grad[l][1] * grad[m][1] +
                                             grad[l][2] * grad[m][2]);
            }
}

/* Vertex coordinates X_{l,i}: bit i of l (voxel units). */
static double vert_coord(int l, int i) { return (double)((l >> i) & 1); }

/* ------------------------------------------------------------------------ */
/* Density filter: rho~_e = sum_i w(x_e - x_i) rho_i / sum_i w(x_e - x_i),    */
/* w(d) = prod_a max(0, r - |d_a|), periodic.  Direct neighborhood sum.       */
/* ------------------------------------------------------------------------ */
static int filter_reach(double r) {
    int R = 0;
    while (r - (double)(R + 1) > 0.0) ++R;
    return R;
}

static double hat(double r, int d) {
    double v = r - fabs((double)d);
    return v > 0.0 ? v : 0.0;
}

void ora_filter(int64_t n, double r, const double *in, double *out) {
    if (!(r > 0.0)) {
        memcpy(out, in, (size_t)(n * n * n) * sizeof(double));
        return;
    }
    const int R = filter_reach(r);
    double wsum = 0.0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) wsum += hat(r, dx) * hat(r, dy) * hat(r, dz);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < n; ++k)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int dz = -R; dz <= R; ++dz)
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx)
                            acc += hat(r, dx) * hat(r, dy) * hat(r, dz) *
                                   in[node_index(i + dx, j + dy, k + dz, n)];
                out[i + n * (j + n * k)] = acc / wsum;
            }
}

/* Transpose of the filter matrix: (F^T y)_i = sum_e F_{e,i} y_e, written as   */
/* the scatter of each element's weighted value onto its neighborhood.        */
void ora_filter_transpose(int64_t n, double r, const double *y, double *out) {
    const int64_t ne = n * n * n;
    if (!(r > 0.0)) {
        memcpy(out, y, (size_t)ne * sizeof(double));
        return;
    }
    const int R = filter_reach(r);
    double wsum = 0.0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) wsum += hat(r, dx) * hat(r, dy) * hat(r, dz);
    memset(out, 0, (size_t)ne * sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                const double ye = y[i + n * (j + n * k)];
                for (int dz = -R; dz <= R; ++dz)
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx)
                            out[node_index(i + dx, j + dy, k + dz, n)] +=
                                hat(r, dx) * hat(r, dy) * hat(r, dz) / wsum * ye;
            }
}

/* SIMP: k_e = kmin + rho~_e^p (k0 - kmin). */
void ora_simp(int64_t ne, const double *rhof, double k0, double kmin, double p, double *k) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) k[e] = kmin + pow(rhof[e], p) * (k0 - kmin);
}

/* ------------------------------------------------------------------------ */
/* Assembly.  Row v has 27 slots, one per neighbor offset (dx,dy,dz) in        */
/* {-1,0,1}^3, slot = (dz+1)*9 + (dy+1)*3 + (dx+1), column = wrapped neighbor. */
/* Entry A[v][u] = sum over elements e containing both v (as vertex l) and u   */
/* (as vertex m) of k_e Khat[l][m].  Requires n >= 3 so the 27 are distinct.   */
/* ------------------------------------------------------------------------ */
void ora_assemble(int64_t n, const double *k, int32_t *cols /* 27*n^3 */, double *vals /* 27*n^3 */) {
    double Kh[64];
    ora_element_matrix(Kh);
    const int64_t nn = n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nn; ++v) {
        const int64_t vi = v % n, vj = (v / n) % n, vk = v / (n * n);
        for (int s = 0; s < 27; ++s) {
            const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
            cols[v * 27 + s] = (int32_t)node_index(vi + dx, vj + dy, vk + dz, n);
            vals[v * 27 + s] = 0.0;
        }
        for (int l = 0; l < 8; ++l) {
            const int la = l & 1, lb = (l >> 1) & 1, lc = (l >> 2) & 1;
            /* element whose local vertex l is v */
            const int64_t e = node_index(vi - la, vj - lb, vk - lc, n);
            for (int m = 0; m < 8; ++m) {
                const int dx = (m & 1) - la, dy = ((m >> 1) & 1) - lb, dz = ((m >> 2) & 1) - lc;
                const int s = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                vals[v * 27 + s] += k[e] * Kh[l * 8 + m];
            }
        }
    }
}

/* Macro loads b^i_v = sum_{e containing v as vertex l} k_e (Khat X)_{l,i}. */
void ora_rhs(int64_t n, const double *k, double *b /* 3*n^3, load-major */) {
    double Kh[64], KX[8][3];
    ora_element_matrix(Kh);
    for (int l = 0; l < 8; ++l)
        for (int i = 0; i < 3; ++i) {
            double acc = 0.0;
            for (int m = 0; m < 8; ++m) acc += Kh[l * 8 + m] * vert_coord(m, i);
            KX[l][i] = acc;
        }
    const int64_t nn = n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nn; ++v) {
        const int64_t vi = v % n, vj = (v / n) % n, vk = v / (n * n);
        double acc[3] = {0, 0, 0};
        for (int l = 0; l < 8; ++l) {
            const int64_t e = node_index(vi - (l & 1), vj - ((l >> 1) & 1), vk - ((l >> 2) & 1), n);
            for (int i = 0; i < 3; ++i) acc[i] += k[e] * KX[l][i];
        }
        for (int i = 0; i < 3; ++i) b[i * nn + v] = acc[i];
    }
}

/* y = A x for one vector, CSR with 27 slots per row. */
void ora_spmv(int64_t nn, const int32_t *cols, const double *vals, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nn; ++v) {
        double acc = 0.0;
        for (int s = 0; s < 27; ++s) acc += vals[v * 27 + s] * x[cols[v * 27 + s]];
        y[v] = acc;
    }
}

static double dot(int64_t nn, const double *a, const double *b) {
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int64_t v = 0; v < nn; ++v) acc += a[v] * b[v];
    return acc;
}

static void remove_mean(int64_t nn, double *x) {
    double m = 0.0;
#pragma omp parallel for reduction(+ : m) schedule(static)
    for (int64_t v = 0; v < nn; ++v) m += x[v];
    m /= (double)nn;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nn; ++v) x[v] -= m;
}

/*
 * Plain conjugate gradients for A x = b on the zero-mean subspace.
 * b is copied and projected to zero mean; x starts at 0; the stop test is the
 * recursive residual ||r|| <= tol ||b||; x is projected to zero mean at exit.
 * out_stats[0] = iterations, [1] = true relative residual ||b - A x||/||b||.
 * Returns 0 when converged, 1 when max_iter was hit.
 */
int ora_cg(int64_t nn, const int32_t *cols, const double *vals, const double *b_in, double tol,
           int64_t max_iter, double *x, double *out_stats) {
    double *b = malloc((size_t)nn * sizeof(double));
    double *r = malloc((size_t)nn * sizeof(double));
    double *p = malloc((size_t)nn * sizeof(double));
    double *q = malloc((size_t)nn * sizeof(double));
    memcpy(b, b_in, (size_t)nn * sizeof(double));
    remove_mean(nn, b);
    const double bnorm = sqrt(dot(nn, b, b));
    int64_t it = 0;
    int status = 0;
    memset(x, 0, (size_t)nn * sizeof(double));
    if (bnorm > 0.0) {
        memcpy(r, b, (size_t)nn * sizeof(double));
        memcpy(p, r, (size_t)nn * sizeof(double));
        double rr = dot(nn, r, r);
        status = 1;
        while (it < max_iter) {
            ora_spmv(nn, cols, vals, p, q);
            const double alpha = rr / dot(nn, p, q);
#pragma omp parallel for schedule(static)
            for (int64_t v = 0; v < nn; ++v) {
                x[v] += alpha * p[v];
                r[v] -= alpha * q[v];
            }
            ++it;
            const double rr_new = dot(nn, r, r);
            if (sqrt(rr_new) <= tol * bnorm) {
                status = 0;
                break;
            }
            const double beta = rr_new / rr;
#pragma omp parallel for schedule(static)
            for (int64_t v = 0; v < nn; ++v) p[v] = r[v] + beta * p[v];
            rr = rr_new;
        }
        remove_mean(nn, x);
    }
    /* true residual */
    ora_spmv(nn, cols, vals, x, q);
    double tr = 0.0;
    for (int64_t v = 0; v < nn; ++v) tr += (b[v] - q[v]) * (b[v] - q[v]);
    out_stats[0] = (double)it;
    out_stats[1] = bnorm > 0.0 ? sqrt(tr) / bnorm : sqrt(tr);
    free(b);
    free(r);
    free(p);
    free(q);
    return status;
}

/* Fixed number of plain CG iterations (no stop test); used to time the oracle */
/* on a bounded sample.  Same arithmetic as ora_cg.                            */
void ora_cg_fixed(int64_t nn, const int32_t *cols, const double *vals, const double *b_in, int64_t iters,
                  double *x) {
    double *r = malloc((size_t)nn * sizeof(double));
    double *p = malloc((size_t)nn * sizeof(double));
    double *q = malloc((size_t)nn * sizeof(double));
    memcpy(r, b_in, (size_t)nn * sizeof(double));
    remove_mean(nn, r);
    memcpy(p, r, (size_t)nn * sizeof(double));
    memset(x, 0, (size_t)nn * sizeof(double));
    double rr = dot(nn, r, r);
    for (int64_t it = 0; it < iters && rr > 0.0; ++it) {
        ora_spmv(nn, cols, vals, p, q);
        const double alpha = rr / dot(nn, p, q);
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < nn; ++v) {
            x[v] += alpha * p[v];
            r[v] -= alpha * q[v];
        }
        const double rr_new = dot(nn, r, r);
        const double beta = rr_new / rr;
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < nn; ++v) p[v] = r[v] + beta * p[v];
        rr = rr_new;
    }
    free(r);
    free(p);
    free(q);
}

/* ------------------------------------------------------------------------ */
/* Element energies E_e,c = (X_i - chi^i_e)^T Khat (X_j - chi^j_e) for the six */
/* pairs c = (0,0),(1,1),(2,2),(0,1),(1,2),(0,2), i.e. [11,22,33,12,23,13].    */
/* ------------------------------------------------------------------------ */
static const int PAIR_I[6] = {0, 1, 2, 0, 1, 0};
static const int PAIR_J[6] = {0, 1, 2, 1, 2, 2};

void ora_energy(int64_t n, const double *chi /* 3*n^3 */, double *E /* 6*n^3, component-major */) {
    double Kh[64];
    ora_element_matrix(Kh);
    const int64_t nn = n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nn; ++e) {
        const int64_t ei = e % n, ej = (e / n) % n, ek = e / (n * n);
        double u[3][8];
        for (int l = 0; l < 8; ++l) {
            const int64_t v = node_index(ei + (l & 1), ej + ((l >> 1) & 1), ek + ((l >> 2) & 1), n);
            for (int i = 0; i < 3; ++i) u[i][l] = vert_coord(l, i) - chi[i * nn + v];
        }
        for (int c = 0; c < 6; ++c) {
            const int i = PAIR_I[c], j = PAIR_J[c];
            double acc = 0.0;
            for (int l = 0; l < 8; ++l)
                for (int m = 0; m < 8; ++m) acc += u[i][l] * Kh[l * 8 + m] * u[j][m];
            E[c * nn + e] = acc;
        }
    }
}

/* kappa_c = N^-3 sum_e k_e E_e,c */
void ora_kappa(int64_t nn, const double *k, const double *E, double *kappa6) {
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int64_t e = 0; e < nn; ++e) acc += k[e] * E[c * nn + e];
        kappa6[c] = acc / (double)nn;
    }
}

/* d g / d rho~_e = sum_c w_c d kappa_c / d rho~_e,                              */
/* d kappa_c / d rho~_e = N^-3 (dk/drho~)(rho~_e) E_e,c, dk/drho~ = p rho~^(p-1) (k0-kmin). */
void ora_sens(int64_t nn, const double *rhof, const double *E, const double *w6, double k0, double kmin,
              double p, double *st) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nn; ++e) {
        double acc = 0.0;
        for (int c = 0; c < 6; ++c) acc += w6[c] * E[c * nn + e];
        st[e] = p * pow(rhof[e], p - 1.0) * (k0 - kmin) * acc / (double)nn;
    }
}

/* ------------------------------------------------------------------------ */
/* Optimality Criteria update with the volume dV/drho_e = N^-3:                */
/*   B_e = max(0, -s_e) / (lambda N^-3),                                       */
/*   rho_new = clamp(rho_e B_e^eta, max(rho_min, rho_e - m), min(1, rho_e + m)) */
/* and lambda found by bisection on [0, 1e9] so that mean(rho_new) = V*.       */
/* Stop when l2 - l1 <= 1e-13 (l1 + l2) or after 200 halvings.                 */
/* ------------------------------------------------------------------------ */
static double oc_value(double rho, double s, double lam, double nn, double move, double eta, double rho_min) {
    const double B = fmax(0.0, -s) * nn / lam;
    const double lo = fmax(rho_min, rho - move);
    const double hi = fmin(1.0, rho + move);
    const double v = rho * pow(B, eta);
    return fmin(hi, fmax(lo, v));
}

double ora_oc_update(int64_t nn, const double *rho, const double *s, double vstar, double move, double eta,
                     double rho_min, double *rho_new, int32_t *steps_out) {
    double l1 = 0.0, l2 = 1e9;
    int steps = 0;
    while (steps < 200 && !((l2 - l1) <= 1e-13 * (l1 + l2))) {
        const double mid = 0.5 * (l1 + l2);
        double vol = 0.0;
#pragma omp parallel for reduction(+ : vol) schedule(static)
        for (int64_t e = 0; e < nn; ++e) vol += oc_value(rho[e], s[e], mid, (double)nn, move, eta, rho_min);
        vol /= (double)nn;
        if (vol > vstar)
            l1 = mid;
        else
            l2 = mid;
        ++steps;
    }
    const double lam = 0.5 * (l1 + l2);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nn; ++e) rho_new[e] = oc_value(rho[e], s[e], lam, (double)nn, move, eta, rho_min);
    if (steps_out) *steps_out = steps;
    return lam;
}
