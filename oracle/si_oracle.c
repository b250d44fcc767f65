/*
 * si_oracle.c -- plain, slow FP64 reference for discrete-ordinates (S_N)
 * source iteration with diamond differencing, 1-D slab and 2-D x-y.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or table with the
 * HIP library.
 *
 * What it computes (arXiv 2509.01416):
 *   * the fixed-source transport equation with isotropic scattering and an
 *     isotropic source, section 5.1 Eq. 12 (1-D) and its x-y analogue;
 *     with weights summing to 1 the emission per unit weight is
 *     Q = sigma_s * phi + q and phi = sum_m w_m psi_m (the scalar flux of
 *     Eq. 17, identical to the paper's, whose weights sum to 2 with a 1/2 on
 *     the emission);
 *   * the model-based iteration M of Eq. 3a/4b realised as S_N source
 *     iteration (section 5.1, text after Eq. 20): phi <- Sweep(sigma_s phi + q);
 *   * the spatial scheme is diamond difference (the paper does not name one):
 *     per direction and cell, with a = 2|mu|/dx, b = 2|eta|/dy,
 *         psi_c = (Q + a psi_in_x + b psi_in_y) / (sigma_t + a + b),
 *         psi_out_x = 2 psi_c - psi_in_x,  psi_out_y = 2 psi_c - psi_in_y;
 *     no negative-flux fix-up, so the discrete system stays linear;
 *   * boundary conditions: vacuum (zero incoming) or reflective (incoming =
 *     the mirrored direction's outgoing value from the previous sweep, i.e.
 *     lagged one iteration).
 *
 * Linearly anisotropic (P1) scattering, section 5.1 Eq. 25: with the first
 * Legendre moment sigma_s1 of the scattering cross section the emission of
 * direction m becomes
 *     Q_m = sigma_s phi + 3 sigma_s1 (mu_m J_x + eta_m J_y) + S,
 *     J = sum_m w_m Omega_m psi_m  (the current; J_y absent in 1-D).
 * In the paper's normalisation (weights summing to 2, the factors 1/2 and
 * 3/2 of Eq. 25) the same emission results.  Source iteration lags J like
 * phi: it comes from the previous sweep (zero before the first).  The P1
 * term integrates to zero over the directions, so particle balance is
 * unchanged.  The sweeps take the anisotropic part as per-cell fields
 * E = 3 sigma_s1 J (NULL: isotropic emission) and return J when asked.
 *
 * Convergence: norm_kind 0 -> ||phi_new - phi_old||_2 / ||phi_new||_2 < tol,
 *              norm_kind 1 -> max_i |phi_new_i - phi_old_i| / |phi_new_i| < tol,
 *              norm_kind 2 -> error bound of the fixed-point iteration: with
 *                r_l the norm of kind 0 and rho = r_l / r_(l-1) the observed
 *                contraction rate, stop once rho < 1 and
 *                r_l * rho / (1 - rho) < tol (a contraction of rate rho
 *                leaves the new iterate within r_l rho / (1 - rho) of the
 *                fixed point, relative to its norm), or r_l = 0.
 *              With a stride K > 1 the same test runs only at iterations
 *                l = K, 2K, ...: r_l is then the relative L2 distance
 *                between phi_l and phi_(l-K) and rho = r_l / r_(l-K) the
 *                contraction over K iterations, and the estimate
 *                r_l rho / (1 - rho) keeps its meaning (the distance of
 *                phi_l to the fixed point for a geometric error).
 * The paper quotes only a tolerance (1e-4, section 5.1); the norms are this
 * library's reading.
 *
 * Face storage (2-D): face[f][k][m], f = 0 x-, 1 x+, 2 y-, 3 y+; k runs along
 * the face (j for x-faces, i for y-faces) up to max(nx, ny); m = direction.
 * After a sweep face[f][k][m] holds the angular flux of direction m on that
 * boundary face (incoming or outgoing).  1-D: face[f][m], f = 0 (x=0), 1 (x=L).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_BAD_ARG -1

/* index of the direction mirrored across a face normal; -1 if absent */
static int mirror_dir(int M, const double *mu, const double *eta, int m,
                      int flip_x) {
    double tm = flip_x ? -mu[m] : mu[m];
    double te = eta ? (flip_x ? eta[m] : -eta[m]) : 0.0;
    for (int k = 0; k < M; ++k) {
        double de = eta ? fabs(eta[k] - te) : 0.0;
        if (fabs(mu[k] - tm) < 1e-12 && de < 1e-12) return k;
    }
    return -1;
}

/* ---------------------------------------------------------------- 2-D --- */

/*
 * One full sweep: every direction, cells in upwind order.
 * face_prev supplies reflective incoming values (may be NULL when no face is
 * reflective); face_out receives all face values (may be NULL).
 * phi must hold nx*ny doubles and is overwritten.  *leak (may be NULL)
 * receives sum_m w_m sum_faces (Omega_m . n) psi_face * face_length.
 */
int or_sweep2d(int nx, int ny, double lx, double ly, int M, const double *mu,
               const double *eta, const double *w, const double *sigma_t,
               const double *emission, const double *ex, const double *ey,
               const int *bc, const double *face_prev, double *face_out,
               double *phi, double *jx, double *jy, double *leak) {
    if (nx <= 0 || ny <= 0 || M <= 0) return OR_BAD_ARG;
    const double dx = lx / nx, dy = ly / ny;
    const int nf = nx > ny ? nx : ny;
    double *ycol = (double *)malloc(sizeof(double) * nx);
    if (!ycol) return OR_BAD_ARG;
    memset(phi, 0, sizeof(double) * nx * ny);
    if (jx) memset(jx, 0, sizeof(double) * nx * ny);
    if (jy) memset(jy, 0, sizeof(double) * nx * ny);
    double lk = 0.0;
    for (int m = 0; m < M; ++m) {
        const double a = 2.0 * fabs(mu[m]) / dx;
        const double b = 2.0 * fabs(eta[m]) / dy;
        const int xpos = mu[m] > 0.0, ypos = eta[m] > 0.0;
        const int fx_in = xpos ? 0 : 1, fx_out = xpos ? 1 : 0;
        const int fy_in = ypos ? 2 : 3, fy_out = ypos ? 3 : 2;
        const int mx = mirror_dir(M, mu, eta, m, 1);
        const int my = mirror_dir(M, mu, eta, m, 0);
        /* incoming y-face values for every column */
        for (int i = 0; i < nx; ++i) {
            double v = 0.0;
            if (bc[fy_in] == 1 && face_prev && my >= 0)
                v = face_prev[((size_t)fy_in * nf + i) * M + my];
            ycol[i] = v;
            if (face_out) face_out[((size_t)fy_in * nf + i) * M + m] = v;
        }
        for (int jj = 0; jj < ny; ++jj) {
            const int j = ypos ? jj : ny - 1 - jj;
            double xin = 0.0;
            if (bc[fx_in] == 1 && face_prev && mx >= 0)
                xin = face_prev[((size_t)fx_in * nf + j) * M + mx];
            if (face_out) face_out[((size_t)fx_in * nf + j) * M + m] = xin;
            lk -= w[m] * fabs(mu[m]) * dy * xin;
            for (int ii = 0; ii < nx; ++ii) {
                const int i = xpos ? ii : nx - 1 - ii;
                const size_t c = (size_t)j * nx + i;
                double q = emission[c];
                if (ex) q += mu[m] * ex[c];
                if (ey) q += eta[m] * ey[c];
                const double psi = (q + a * xin + b * ycol[i]) /
                                   (sigma_t[c] + a + b);
                xin = 2.0 * psi - xin;
                ycol[i] = 2.0 * psi - ycol[i];
                phi[c] += w[m] * psi;
                if (jx) jx[c] += w[m] * mu[m] * psi;
                if (jy) jy[c] += w[m] * eta[m] * psi;
            }
            if (face_out) face_out[((size_t)fx_out * nf + j) * M + m] = xin;
            lk += w[m] * fabs(mu[m]) * dy * xin;
        }
        for (int i = 0; i < nx; ++i) {
            if (face_out) face_out[((size_t)fy_out * nf + i) * M + m] = ycol[i];
            lk += w[m] * fabs(eta[m]) * dx * ycol[i];
        }
        /* the incoming y contribution */
        if (bc[fy_in] == 1 && face_prev && my >= 0)
            for (int i = 0; i < nx; ++i)
                lk -= w[m] * fabs(eta[m]) * dx *
                      face_prev[((size_t)fy_in * nf + i) * M + my];
    }
    free(ycol);
    if (leak) *leak = lk;
    return OR_OK;
}

static double change_norm(size_t n, const double *a, const double *b,
                          int kind) {
    if (kind == 1) {
        double r = 0.0;
        for (size_t i = 0; i < n; ++i) {
            double d = fabs(a[i] - b[i]);
            double s = fabs(a[i]);
            double q = s > 0.0 ? d / s : (d > 0.0 ? INFINITY : 0.0);
            if (q > r) r = q;
        }
        return r;
    }
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double d = a[i] - b[i];
        num += d * d;
        den += a[i] * a[i];
    }
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return sqrt(num / den);
}

/* Stopping test of one iteration: r = change norm of this iteration (kind 0
 * or 1 as computed by change_norm; kind 2 uses the L2 norm), r_prev = that of
 * the previous iteration (INFINITY before the second). */
static int converged(double r, double r_prev, double tol, int kind) {
    if (kind != 2) return r < tol;
    if (r == 0.0) return 1;
    if (!(r_prev < INFINITY) || !(r_prev > 0.0)) return 0;
    const double rho = r / r_prev;
    if (!(rho < 1.0)) return 0;
    return r * rho / (1.0 - rho) < tol;
}

/*
 * Source iteration to tolerance.  phi0 may be NULL (zero start).  With a
 * warm start, reflective faces start isotropic at the adjacent cell's phi0.
 * stats[0] iterations, [1] last change norm, [2] leakage of the last sweep,
 * [3] sum sigma_s (phi_new - phi_old) V of the last iteration.
 * hist (may be NULL) receives the change norm of every iteration.
 */
int or_si2d(int nx, int ny, double lx, double ly, int M, const double *mu,
            const double *eta, const double *w, const double *sigma_t,
            const double *sigma_s, const double *sigma_s1, const double *q, const int *bc,
            const double *phi0, double tol, int max_iter, int norm_kind,
            int stride, double *phi, double *stats, double *hist) {
    if (nx <= 0 || ny <= 0 || M <= 0 || max_iter <= 0 || stride <= 0) return OR_BAD_ARG;
    const size_t n = (size_t)nx * ny;
    const int nf = nx > ny ? nx : ny;
    const size_t fsz = (size_t)4 * nf * M;
    double *Q = (double *)malloc(sizeof(double) * n);
    double *phin = (double *)malloc(sizeof(double) * n);
    double *fa = (double *)calloc(fsz, sizeof(double));
    double *fb = (double *)calloc(fsz, sizeof(double));
    double *snap = (double *)malloc(sizeof(double) * n);
    /* P1: E = 3 sigma_s1 J of the previous sweep (x, y), the new J */
    double *ex = sigma_s1 ? (double *)calloc(4 * n, sizeof(double)) : NULL;
    double *ey = ex ? ex + n : NULL, *jx = ex ? ex + 2 * n : NULL, *jy = ex ? ex + 3 * n : NULL;
    if (!Q || !phin || !fa || !fb || !snap || (sigma_s1 && !ex)) {
        free(Q); free(phin); free(fa); free(fb); free(snap); free(ex);
        return OR_BAD_ARG;
    }
    if (norm_kind != 2) stride = 1;
    if (phi0) {
        memcpy(phi, phi0, sizeof(double) * n);
        for (int m = 0; m < M; ++m) {
            for (int j = 0; j < ny; ++j) {
                fa[((size_t)0 * nf + j) * M + m] = phi0[(size_t)j * nx];
                fa[((size_t)1 * nf + j) * M + m] = phi0[(size_t)j * nx + nx - 1];
            }
            for (int i = 0; i < nx; ++i) {
                fa[((size_t)2 * nf + i) * M + m] = phi0[i];
                fa[((size_t)3 * nf + i) * M + m] = phi0[(size_t)(ny - 1) * nx + i];
            }
        }
    } else {
        memset(phi, 0, sizeof(double) * n);
    }
    memcpy(snap, phi, sizeof(double) * n);
    const double V = (lx / nx) * (ly / ny);
    int status = OR_NOT_CONVERGED, it = 0;
    double r = INFINITY, r_prev = INFINITY, r_step = INFINITY, leak = 0.0, dscat = 0.0;
    for (it = 1; it <= max_iter; ++it) {
        for (size_t c = 0; c < n; ++c) Q[c] = sigma_s[c] * phi[c] + q[c];
        or_sweep2d(nx, ny, lx, ly, M, mu, eta, w, sigma_t, Q, ex, ey, bc, fa, fb,
                   phin, jx, jy, &leak);
        if (sigma_s1)
            for (size_t c = 0; c < n; ++c) {
                ex[c] = 3.0 * sigma_s1[c] * jx[c];
                ey[c] = 3.0 * sigma_s1[c] * jy[c];
            }
        r_step = change_norm(n, phin, phi, norm_kind == 1);
        dscat = 0.0;
        for (size_t c = 0; c < n; ++c) dscat += sigma_s[c] * (phin[c] - phi[c]) * V;
        memcpy(phi, phin, sizeof(double) * n);
        double *t = fa; fa = fb; fb = t;
        if (hist) hist[it - 1] = r_step;
        if (it % stride != 0) continue;
        r_prev = r;
        r = stride == 1 ? r_step : change_norm(n, phin, snap, 0);
        memcpy(snap, phin, sizeof(double) * n);
        if (converged(r, r_prev, tol, norm_kind)) { status = OR_OK; break; }
    }
    if (it > max_iter) it = max_iter;
    if (stats) {
        stats[0] = it; stats[1] = r; stats[2] = leak; stats[3] = dscat;
    }
    free(Q); free(phin); free(fa); free(fb); free(snap); free(ex);
    return status;
}

/* ---------------------------------------------------------------- 1-D --- */

/* One 1-D sweep; face layout face[f][m], f = 0 left, 1 right. */
int or_sweep1d(int nx, double lx, int M, const double *mu, const double *w,
               const double *sigma_t, const double *emission, const double *ex,
               const int *bc, const double *face_prev, double *face_out,
               double *phi, double *jx, double *leak) {
    if (nx <= 0 || M <= 0) return OR_BAD_ARG;
    const double dx = lx / nx;
    memset(phi, 0, sizeof(double) * nx);
    if (jx) memset(jx, 0, sizeof(double) * nx);
    double lk = 0.0;
    for (int m = 0; m < M; ++m) {
        const double a = 2.0 * fabs(mu[m]) / dx;
        const int pos = mu[m] > 0.0;
        const int fin = pos ? 0 : 1, fout = pos ? 1 : 0;
        const int mm = mirror_dir(M, mu, NULL, m, 1);
        double in = 0.0;
        if (bc[fin] == 1 && face_prev && mm >= 0) in = face_prev[fin * M + mm];
        if (face_out) face_out[fin * M + m] = in;
        lk -= w[m] * fabs(mu[m]) * in;
        for (int ii = 0; ii < nx; ++ii) {
            const int i = pos ? ii : nx - 1 - ii;
            const double qm = ex ? emission[i] + mu[m] * ex[i] : emission[i];
            const double psi = (qm + a * in) / (sigma_t[i] + a);
            in = 2.0 * psi - in;
            phi[i] += w[m] * psi;
            if (jx) jx[i] += w[m] * mu[m] * psi;
        }
        if (face_out) face_out[fout * M + m] = in;
        lk += w[m] * fabs(mu[m]) * in;
    }
    if (leak) *leak = lk;
    return OR_OK;
}

int or_si1d(int nx, double lx, int M, const double *mu, const double *w,
            const double *sigma_t, const double *sigma_s, const double *sigma_s1,
            const double *q,
            const int *bc, const double *phi0, double tol, int max_iter,
            int norm_kind, int stride, double *phi, double *stats, double *hist) {
    if (nx <= 0 || M <= 0 || max_iter <= 0 || stride <= 0) return OR_BAD_ARG;
    double *Q = (double *)malloc(sizeof(double) * nx);
    double *phin = (double *)malloc(sizeof(double) * nx);
    double *fa = (double *)calloc((size_t)2 * M, sizeof(double));
    double *fb = (double *)calloc((size_t)2 * M, sizeof(double));
    double *snap = (double *)malloc(sizeof(double) * nx);
    double *ex = sigma_s1 ? (double *)calloc(2 * (size_t)nx, sizeof(double)) : NULL;
    double *jx = ex ? ex + nx : NULL;
    if (!Q || !phin || !fa || !fb || !snap || (sigma_s1 && !ex)) {
        free(Q); free(phin); free(fa); free(fb); free(snap); free(ex);
        return OR_BAD_ARG;
    }
    if (norm_kind != 2) stride = 1;
    if (phi0) {
        memcpy(phi, phi0, sizeof(double) * nx);
        for (int m = 0; m < M; ++m) {
            fa[m] = phi0[0];
            fa[M + m] = phi0[nx - 1];
        }
    } else {
        memset(phi, 0, sizeof(double) * nx);
    }
    memcpy(snap, phi, sizeof(double) * nx);
    const double V = lx / nx;
    int status = OR_NOT_CONVERGED, it;
    double r = INFINITY, r_prev = INFINITY, r_step = INFINITY, leak = 0.0, dscat = 0.0;
    for (it = 1; it <= max_iter; ++it) {
        for (int c = 0; c < nx; ++c) Q[c] = sigma_s[c] * phi[c] + q[c];
        or_sweep1d(nx, lx, M, mu, w, sigma_t, Q, ex, bc, fa, fb, phin, jx, &leak);
        if (sigma_s1)
            for (int c = 0; c < nx; ++c) ex[c] = 3.0 * sigma_s1[c] * jx[c];
        r_step = change_norm((size_t)nx, phin, phi, norm_kind == 1);
        dscat = 0.0;
        for (int c = 0; c < nx; ++c) dscat += sigma_s[c] * (phin[c] - phi[c]) * V;
        memcpy(phi, phin, sizeof(double) * nx);
        double *t = fa; fa = fb; fb = t;
        if (hist) hist[it - 1] = r_step;
        if (it % stride != 0) continue;
        r_prev = r;
        r = stride == 1 ? r_step : change_norm((size_t)nx, phin, snap, 0);
        memcpy(snap, phin, sizeof(double) * nx);
        if (converged(r, r_prev, tol, norm_kind)) { status = OR_OK; break; }
    }
    if (it > max_iter) it = max_iter;
    if (stats) {
        stats[0] = it; stats[1] = r; stats[2] = leak; stats[3] = dscat;
    }
    free(Q); free(phin); free(fa); free(fb); free(snap); free(ex);
    return status;
}
