/*
 * FP64 CPU oracle of the volume-rendering hot path (features + raymarch + reverse mode).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or helper with the GPU
 * library: it is written directly from the paper's equations and from the readings of its silent
 * or garbled points that the design notes list.  Everything is IEEE double, no fast-math, no
 * FMA contraction (built with -ffp-contract=off), OpenMP only over independent voxels/rays.
 *
 * Paper: "Decentralized Direct Volume Rendering: A Browser-Native GPU Architecture for MRI
 * Digital Twins in Resource-Constrained Settings".
 *   Sec. 2.2 Eq. 1   min-max normalization
 *   Sec. 2.3 Eq. 2   central-difference gradient with voxel spacing h
 *   Sec. 2.3 Eq. 3   directional curvature k = g^T H g / g^T g   (Hessian at the first scale)
 *   Sec. 1           "multi-scale Hessian analysis and vesselness measures" (Frangi et al. 1998)
 *   Sec. 2.4 Eq. 4   opacity = f(I) * |grad I| / |grad I|_max * w(k), clamped to [0, 1]
 *   Sec. 2.4 Eq. 5-6 front-to-back emission-absorption compositing
 *
 * Grid: voxel (i,j,k) holds I[k][j][i] at (i*hx, j*hy, k*hz) mm; arrays are C order, x fastest.
 * Index clamping ("clamp to edge") is used wherever a stencil leaves the grid.
 *
 * Parity pins (checked by the CPU tests): closed forms (linear ramp, quadratic bowl, Gaussian
 * tube, Beer-Lambert slab, partial-volume slab, homogeneous column), library special cases
 * (scipy gaussian_filter, numpy eigvalsh, scipy map_coordinates, numpy interp), NumPy brute force
 * on tiny volumes, and central finite differences for the reverse mode.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, k) ((int64_t)(k) * ny * nx + (int64_t)(j) * nx + (int64_t)(i))

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------------------------ */
/* Eq. 1: global min-max normalization; a constant volume maps to 0.                            */
int oracle_normalize(const double *raw, int64_t n, double *out, double *mn_out, double *mx_out)
{
    if (n <= 0) return -1;
    double mn = raw[0], mx = raw[0];
    for (int64_t i = 1; i < n; ++i) {
        if (raw[i] < mn) mn = raw[i];
        if (raw[i] > mx) mx = raw[i];
    }
    for (int64_t i = 0; i < n; ++i) out[i] = (mx > mn) ? (raw[i] - mn) / (mx - mn) : 0.0;
    if (mn_out) *mn_out = mn;
    if (mx_out) *mx_out = mx;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Eq. 2: g_a = (I[a+1] - I[a-1]) / (2 h_a), indices clamped to the grid.  gmax = max |g|_2      */
/* (the |grad I|_max of Eq. 4, a global reduction).  g is planar [3][nz][ny][nx].                */
int oracle_gradient(const double *I, int nx, int ny, int nz, double hx, double hy, double hz,
                    double *g, double *gmax_out)
{
    if (nx < 2 || ny < 2 || nz < 2) return -1;
    const int64_t N = (int64_t)nx * ny * nz;
    double gmax = 0.0;
#pragma omp parallel for collapse(2) reduction(max : gmax)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t c = IDX(i, j, k);
                double gx = (I[IDX(clampi(i + 1, 0, nx - 1), j, k)] - I[IDX(clampi(i - 1, 0, nx - 1), j, k)]) / (2.0 * hx);
                double gy = (I[IDX(i, clampi(j + 1, 0, ny - 1), k)] - I[IDX(i, clampi(j - 1, 0, ny - 1), k)]) / (2.0 * hy);
                double gz = (I[IDX(i, j, clampi(k + 1, 0, nz - 1))] - I[IDX(i, j, clampi(k - 1, 0, nz - 1))]) / (2.0 * hz);
                g[c] = gx;
                g[N + c] = gy;
                g[2 * N + c] = gz;
                double m = sqrt(gx * gx + gy * gy + gz * gz);
                if (m > gmax) gmax = m;
            }
    *gmax_out = gmax;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Gaussian scale space: sampled Gaussian exp(-j^2 / (2 s^2)), j = -r..r with r = floor(3 s + 1/2) */
/* (at least 1), normalized to unit sum; applied along x, then y, then z with clamped indices.   */
int oracle_gauss_radius(double sigma_vox) { int r = (int)floor(3.0 * sigma_vox + 0.5); return r < 1 ? 1 : r; }

static double *gauss_weights(double sigma_vox, int *r_out)
{
    int r = oracle_gauss_radius(sigma_vox);
    double *w = (double *)malloc(sizeof(double) * (2 * r + 1));
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) { w[j + r] = exp(-(double)j * j / (2.0 * sigma_vox * sigma_vox)); sum += w[j + r]; }
    for (int j = 0; j <= 2 * r; ++j) w[j] /= sum;
    *r_out = r;
    return w;
}

int oracle_smooth(const double *I, int nx, int ny, int nz, double sx, double sy, double sz, double *s)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double *tmp = (double *)malloc(sizeof(double) * N);
    if (!tmp) return -2;
    int rx, ry, rz;
    double *wx = gauss_weights(sx, &rx), *wy = gauss_weights(sy, &ry), *wz = gauss_weights(sz, &rz);
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int t = -rx; t <= rx; ++t) acc += wx[t + rx] * I[IDX(clampi(i + t, 0, nx - 1), j, k)];
                s[IDX(i, j, k)] = acc;
            }
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int t = -ry; t <= ry; ++t) acc += wy[t + ry] * s[IDX(i, clampi(j + t, 0, ny - 1), k)];
                tmp[IDX(i, j, k)] = acc;
            }
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int t = -rz; t <= rz; ++t) acc += wz[t + rz] * tmp[IDX(i, j, clampi(k + t, 0, nz - 1))];
                s[IDX(i, j, k)] = acc;
            }
    free(tmp); free(wx); free(wy); free(wz);
    return 0;
}

/* Hessian of the smoothed field by central second differences (indices clamped):              */
/* H_aa = (s[+1] - 2 s + s[-1]) / h_a^2, H_ab = (s[+,+] - s[+,-] - s[-,+] + s[-,-]) / (4 h_a h_b). */
/* Order of the 6 entries: xx, yy, zz, xy, xz, yz.                                              */
static void hessian_at(const double *s, int nx, int ny, int nz, double hx, double hy, double hz,
                       int i, int j, int k, double H[6])
{
    const int ip = (int)clampi(i + 1, 0, nx - 1), im = (int)clampi(i - 1, 0, nx - 1);
    const int jp = (int)clampi(j + 1, 0, ny - 1), jm = (int)clampi(j - 1, 0, ny - 1);
    const int kp = (int)clampi(k + 1, 0, nz - 1), km = (int)clampi(k - 1, 0, nz - 1);
    const double c = s[IDX(i, j, k)];
    H[0] = (s[IDX(ip, j, k)] - 2.0 * c + s[IDX(im, j, k)]) / (hx * hx);
    H[1] = (s[IDX(i, jp, k)] - 2.0 * c + s[IDX(i, jm, k)]) / (hy * hy);
    H[2] = (s[IDX(i, j, kp)] - 2.0 * c + s[IDX(i, j, km)]) / (hz * hz);
    H[3] = (s[IDX(ip, jp, k)] - s[IDX(ip, jm, k)] - s[IDX(im, jp, k)] + s[IDX(im, jm, k)]) / (4.0 * hx * hy);
    H[4] = (s[IDX(ip, j, kp)] - s[IDX(ip, j, km)] - s[IDX(im, j, kp)] + s[IDX(im, j, km)]) / (4.0 * hx * hz);
    H[5] = (s[IDX(i, jp, kp)] - s[IDX(i, jp, km)] - s[IDX(i, jm, kp)] + s[IDX(i, jm, km)]) / (4.0 * hy * hz);
}

int oracle_hessian(const double *s, int nx, int ny, int nz, double hx, double hy, double hz, double *H)
{
    const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double h6[6];
                hessian_at(s, nx, ny, nz, hx, hy, hz, i, j, k, h6);
                for (int e = 0; e < 6; ++e) H[e * N + IDX(i, j, k)] = h6[e];
            }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations (a method deliberately      */
/* different from the closed-form trigonometric solver of the GPU path).  A = xx,yy,zz,xy,xz,yz.  */
/* Output sorted by (|lambda|, lambda) ascending: lam[0] = lambda1 (smallest magnitude).         */
static void jacobi3(double a[3][3], double d[3])
{
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = a[p][q];
                if (apq == 0.0) continue;
                double diag = fabs(a[p][p]) + fabs(a[q][q]);
                /* below resolution of the diagonal: drop it (standard Jacobi convergence rule) */
                if (sweep > 4 && fabs(apq) * 1e18 < diag) { a[p][q] = a[q][p] = 0.0; continue; }
                double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150) t = 1.0 / (2.0 * theta);
                else t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* rotate rows/cols p and q: A' = J^T A J zeroes a[p][q] */
                a[p][p] -= t * apq;
                a[q][q] += t * apq;
                a[p][q] = a[q][p] = 0.0;
                for (int r = 0; r < 3; ++r) {
                    if (r == p || r == q) continue;
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = a[p][r] = c * arp - s * arq;
                    a[r][q] = a[q][r] = s * arp + c * arq;
                }
            }
    }
    d[0] = a[0][0]; d[1] = a[1][1]; d[2] = a[2][2];
}

static int mag_less(double a, double b) { return fabs(a) < fabs(b) || (fabs(a) == fabs(b) && a < b); }

void oracle_eig3(const double A[6], double lam[3])
{
    double a[3][3] = {{A[0], A[3], A[4]}, {A[3], A[1], A[5]}, {A[4], A[5], A[2]}};
    jacobi3(a, lam);
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2 - x; ++y)
            if (mag_less(lam[y + 1], lam[y])) { double t = lam[y]; lam[y] = lam[y + 1]; lam[y + 1] = t; }
}

/* Frangi vesselness for bright tubes on magnitude-sorted eigenvalues of the scale-normalized    */
/* Hessian: 0 unless lambda2 < 0 and lambda3 < 0; else                                            */
/* (1 - exp(-Ra^2/2a^2)) exp(-Rb^2/2b^2) (1 - exp(-S^2/2c^2)), Ra = |l2|/|l3|,                     */
/* Rb = |l1|/sqrt(|l2 l3|), S^2 = l1^2 + l2^2 + l3^2.                                              */
double oracle_vesselness(const double lam[3], double alpha, double beta, double c)
{
    double l1 = lam[0], l2 = lam[1], l3 = lam[2];
    if (l2 >= 0.0 || l3 >= 0.0) return 0.0;
    double Ra = fabs(l2) / fabs(l3);
    double Rb = fabs(l1) / sqrt(fabs(l2 * l3));
    double S2 = l1 * l1 + l2 * l2 + l3 * l3;
    return (1.0 - exp(-Ra * Ra / (2.0 * alpha * alpha))) * exp(-Rb * Rb / (2.0 * beta * beta)) *
           (1.0 - exp(-S2 / (2.0 * c * c)));
}

/* Eq. 3: k = g^T H g / g^T g with H at the first scale (unnormalized, I/mm^2) and the Eq. 2     */
/* gradient; g is scaled by its largest component first; k = 0 exactly where g = 0.               */
static double curvature(const double g[3], const double H[6])
{
    double m = fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2])));
    if (m == 0.0) return 0.0;
    double u0 = g[0] / m, u1 = g[1] / m, u2 = g[2] / m;
    double num = H[0] * u0 * u0 + H[1] * u1 * u1 + H[2] * u2 * u2 +
                 2.0 * (H[3] * u0 * u1 + H[4] * u0 * u2 + H[5] * u1 * u2);
    return num / (u0 * u0 + u1 * u1 + u2 * u2);
}

/* Full feature pass.  sigma_mm[s] are the scales in mm (per-axis sigma_a = sigma / h_a).        */
/* c <= 0 selects Frangi's rule c = 1/2 max over voxels and scales of |sigma^2 H|_F.             */
/* Optional outputs: H0 [6][N] at the first scale, lam [nsigma][3][N] (sorted eigenvalues of     */
/* sigma^2 H), Vs [nsigma][N] per-scale vesselness.                                              */
int oracle_features(const double *I, int nx, int ny, int nz, double hx, double hy, double hz,
                    int nsigma, const double *sigma_mm, double alpha, double beta, double c,
                    double *g, double *kappa, double *V, double *gmax, double *c_used,
                    double *H0, double *lam, double *Vs)
{
    if (nx < 2 || ny < 2 || nz < 2 || nsigma < 1 || hx <= 0 || hy <= 0 || hz <= 0) return -1;
    const int64_t N = (int64_t)nx * ny * nz;
    int rc = oracle_gradient(I, nx, ny, nz, hx, hy, hz, g, gmax);
    if (rc) return rc;
    double *s = (double *)malloc(sizeof(double) * N);
    if (!s) return -2;

    if (c <= 0.0) {
        double fro = 0.0;
        for (int sc = 0; sc < nsigma; ++sc) {
            const double sg = sigma_mm[sc];
            oracle_smooth(I, nx, ny, nz, sg / hx, sg / hy, sg / hz, s);
#pragma omp parallel for collapse(2) reduction(max : fro)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        double H[6];
                        hessian_at(s, nx, ny, nz, hx, hy, hz, i, j, k, H);
                        double f = 0.0;
                        for (int e = 0; e < 6; ++e) f += (e < 3 ? 1.0 : 2.0) * (sg * sg * H[e]) * (sg * sg * H[e]);
                        f = sqrt(f);
                        if (f > fro) fro = f;
                    }
        }
        c = 0.5 * fro;
        if (c == 0.0) c = 1.0; /* flat volume: every S is 0 and V is 0 whatever c is */
    }
    if (c_used) *c_used = c;

    for (int64_t v = 0; v < N; ++v) V[v] = 0.0;
    for (int sc = 0; sc < nsigma; ++sc) {
        const double sg = sigma_mm[sc];
        oracle_smooth(I, nx, ny, nz, sg / hx, sg / hy, sg / hz, s);
#pragma omp parallel for collapse(2)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const int64_t v = IDX(i, j, k);
                    double H[6];
                    hessian_at(s, nx, ny, nz, hx, hy, hz, i, j, k, H);
                    if (sc == 0) {
                        double gv[3] = {g[v], g[N + v], g[2 * N + v]};
                        kappa[v] = curvature(gv, H);
                        if (H0) for (int e = 0; e < 6; ++e) H0[e * N + v] = H[e];
                    }
                    double A[6], l[3];
                    for (int e = 0; e < 6; ++e) A[e] = sg * sg * H[e];
                    oracle_eig3(A, l);
                    if (lam) for (int e = 0; e < 3; ++e) lam[((int64_t)sc * 3 + e) * N + v] = l[e];
                    double vs = oracle_vesselness(l, alpha, beta, c);
                    if (Vs) Vs[(int64_t)sc * N + v] = vs;
                    if (vs > V[v]) V[v] = vs;
                }
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Raymarch.  Camera record (16 doubles): persp, width, height, o[3], d0[3], du[3], dv[3], pad.   */
/* ortho: origin o + (i+1/2) du + (j+1/2) dv, direction d0;  persp: origin o, direction          */
/* normalize(d0 + (i+1/2) du + (j+1/2) dv).  Render params (6 doubles): lambda_g, lambda_k,       */
/* kappa0, lambda_v, step_vox, et_alpha.                                                          */

typedef struct {
    const double *I, *g, *kap, *ves;
    int nx, ny, nz;
    double h[3], gmax;
    int K;
    const double *knots, *rgba;
    double lg, lk, k0, lv, step, et;
} scene_t;

typedef struct { int64_t idx[8]; double w[8]; } corners_t;

/* Ray against the box [0,(n-1)h] (slab method).  Returns 0 for a miss. */
static int make_ray(const scene_t *sc, const double *cam, int pi, int pj, double o[3], double d[3],
                    double *tn, double *tf)
{
    const double fi = pi + 0.5, fj = pj + 0.5;
    if (cam[0] != 0.0) {
        double n2 = 0.0;
        for (int a = 0; a < 3; ++a) { o[a] = cam[3 + a]; d[a] = cam[6 + a] + fi * cam[9 + a] + fj * cam[12 + a]; n2 += d[a] * d[a]; }
        double n = sqrt(n2);
        for (int a = 0; a < 3; ++a) d[a] /= n;
    } else {
        for (int a = 0; a < 3; ++a) { o[a] = cam[3 + a] + fi * cam[9 + a] + fj * cam[12 + a]; d[a] = cam[6 + a]; }
    }
    const int n[3] = {sc->nx, sc->ny, sc->nz};
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double lo = 0.0, hi = (n[a] - 1) * sc->h[a];
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return 0;
            continue;
        }
        double ta = (lo - o[a]) / d[a], tb = (hi - o[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    *tn = t0 > 0.0 ? t0 : 0.0;
    *tf = t1;
    return *tf > *tn;
}

/* Trilinear interpolation at p (mm): q = p/h clamped to [0, n-1], cell i0 = min(floor q, n-2). */
static void sample(const scene_t *sc, const double p[3], double *I, double gv[3], double *kap, double *ves,
                   corners_t *cn)
{
    const int n[3] = {sc->nx, sc->ny, sc->nz};
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double q = p[a] / sc->h[a];
        if (q < 0.0) q = 0.0;
        if (q > n[a] - 1) q = n[a] - 1;
        int c = (int)floor(q);
        if (c > n[a] - 2) c = n[a] - 2;
        i0[a] = c;
        f[a] = q - c;
    }
    const int nx = sc->nx, ny = sc->ny;
    const int64_t N = (int64_t)sc->nx * sc->ny * sc->nz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int e = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx, ++e) {
                const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                const int64_t v = IDX(i0[0] + dx, i0[1] + dy, i0[2] + dz);
                acc[0] += w * sc->I[v];
                acc[1] += w * sc->g[v];
                acc[2] += w * sc->g[N + v];
                acc[3] += w * sc->g[2 * N + v];
                acc[4] += w * sc->kap[v];
                acc[5] += w * sc->ves[v];
                if (cn) { cn->idx[e] = v; cn->w[e] = w; }
            }
    *I = acc[0]; gv[0] = acc[1]; gv[1] = acc[2]; gv[2] = acc[3]; *kap = acc[4]; *ves = acc[5];
}

/* Piecewise-linear TF: segment i with x_i <= I < x_{i+1}; clamped to the end values outside.   */
/* Returns the segment (-1 below, K-1 at or above the last knot), t on it, values and slopes.    */
static int tf_eval(const scene_t *sc, double I, double v[4], double dv[4], double *t_out)
{
    const int K = sc->K;
    const double *x = sc->knots, *c = sc->rgba;
    if (I < x[0]) { for (int ch = 0; ch < 4; ++ch) { v[ch] = c[ch]; dv[ch] = 0.0; } *t_out = 0.0; return -1; }
    if (I >= x[K - 1]) { for (int ch = 0; ch < 4; ++ch) { v[ch] = c[4 * (K - 1) + ch]; dv[ch] = 0.0; } *t_out = 0.0; return K - 1; }
    int i = 0;
    while (!(x[i] <= I && I < x[i + 1])) ++i;
    const double wdt = x[i + 1] - x[i], t = (I - x[i]) / wdt;
    for (int ch = 0; ch < 4; ++ch) {
        v[ch] = (1.0 - t) * c[4 * i + ch] + t * c[4 * (i + 1) + ch];
        dv[ch] = (c[4 * (i + 1) + ch] - c[4 * i + ch]) / wdt;
    }
    *t_out = t;
    return i;
}

/* One sample's optical state (Eq. 4 with the extinction reading): sigma_s = tau * m * w * u,   */
/* m = (1-lg) + lg min(|g|/gmax, 1), w = (1-lk) + lk |k| / (|k| + k0), u = 1 + lv V,            */
/* x = sigma_s delta_k, alpha = 1 - exp(-x).                                                     */
typedef struct {
    double alpha, x, M, dk, T, c[3], v[4], dv[4], t;
    double gv[3], gn, kap, m, w, u; /* interpolated features and the three factors of M */
    int seg;
    corners_t cn;
} samp_t;

static void shade(const scene_t *sc, const double p[3], double dk, samp_t *s, int want_corners)
{
    double I, gv[3], kap, ves;
    sample(sc, p, &I, gv, &kap, &ves, want_corners ? &s->cn : NULL);
    s->seg = tf_eval(sc, I, s->v, s->dv, &s->t);
    const double gn = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
    const double m = (sc->gmax > 0.0) ? (1.0 - sc->lg) + sc->lg * fmin(gn / sc->gmax, 1.0) : (1.0 - sc->lg);
    const double ak = fabs(kap);
    const double w = (1.0 - sc->lk) + sc->lk * ak / (ak + sc->k0);
    const double u = 1.0 + sc->lv * ves;
    s->M = m * w * u;
    s->m = m; s->w = w; s->u = u;
    s->gv[0] = gv[0]; s->gv[1] = gv[1]; s->gv[2] = gv[2]; s->gn = gn; s->kap = kap;
    s->dk = dk;
    s->x = s->v[3] * s->M * dk;
    s->alpha = -expm1(-s->x);
    s->c[0] = s->v[0]; s->c[1] = s->v[1]; s->c[2] = s->v[2];
}

/* Segments: delta = step * min h, L = tf - tn, N = ceil(L / delta); delta_k = delta except the   */
/* last, L - (N-1) delta.  Sample k sits at the segment midpoint tn + k delta + delta_k / 2.      */
static int64_t march(const scene_t *sc, const double o[3], const double d[3], double tn, double tf,
                     samp_t *buf, int64_t cap, double out[4], double *T_last, int32_t *k_last, int want_corners)
{
    const double hmin = fmin(sc->h[0], fmin(sc->h[1], sc->h[2]));
    const double delta = sc->step * hmin;
    const double L = tf - tn;
    const int64_t Nseg = (int64_t)ceil(L / delta);
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t k = 0, last = -1;
    double Tprev = 1.0;
    for (k = 0; k < Nseg; ++k) {
        const double dk = (k < Nseg - 1) ? delta : L - (double)(Nseg - 1) * delta;
        const double tk = tn + (double)k * delta + 0.5 * dk;
        double p[3] = {o[0] + tk * d[0], o[1] + tk * d[1], o[2] + tk * d[2]};
        samp_t s;
        shade(sc, p, dk, &s, want_corners);
        s.T = T;
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * s.alpha * s.c[ch];
        Tprev = T;
        T = T * exp(-s.x);
        last = k;
        if (buf && k < cap) buf[k] = s;
        if (sc->et > 0.0 && T <= 1.0 - sc->et) break;
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    *T_last = Tprev;
    *k_last = (int32_t)last;
    return last + 1;
}

static void scene_init(scene_t *sc, const double *I, const double *g, const double *kap, const double *ves,
                       int nx, int ny, int nz, double hx, double hy, double hz, double gmax,
                       int K, const double *knots, const double *rgba, const double *prm)
{
    sc->I = I; sc->g = g; sc->kap = kap; sc->ves = ves;
    sc->nx = nx; sc->ny = ny; sc->nz = nz;
    sc->h[0] = hx; sc->h[1] = hy; sc->h[2] = hz; sc->gmax = gmax;
    sc->K = K; sc->knots = knots; sc->rgba = rgba;
    sc->lg = prm[0]; sc->lk = prm[1]; sc->k0 = prm[2]; sc->lv = prm[3]; sc->step = prm[4]; sc->et = prm[5];
}

/* Render the listed pixels: pix[p] = (camera, i, j).  out [npix][4] = premultiplied (R,G,B), A.  */
/* T_last = transmittance before the last evaluated sample, k_last = its index (-1 on a miss).    */
int oracle_render(const double *I, const double *g, const double *kap, const double *ves,
                  int nx, int ny, int nz, double hx, double hy, double hz, double gmax,
                  int K, const double *knots, const double *rgba, const double *prm,
                  const double *cams, int ncam, const int32_t *pix, int64_t npix,
                  double *out, double *T_last, int32_t *k_last, int64_t *nsamp)
{
    if (nx < 2 || ny < 2 || nz < 2 || K < 2) return -1;
    scene_t sc;
    scene_init(&sc, I, g, kap, ves, nx, ny, nz, hx, hy, hz, gmax, K, knots, rgba, prm);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t p = 0; p < npix; ++p) {
        const int cid = pix[3 * p];
        double o[3], d[3], tn, tf, px[4] = {0, 0, 0, 0}, Tl = 1.0;
        int32_t kl = -1;
        if (cid >= 0 && cid < ncam && make_ray(&sc, cams + 16 * cid, pix[3 * p + 1], pix[3 * p + 2], o, d, &tn, &tf))
            total += march(&sc, o, d, tn, tf, NULL, 0, px, &Tl, &kl, 0);
        for (int ch = 0; ch < 4; ++ch) out[4 * p + ch] = px[ch];
        if (T_last) T_last[p] = Tl;
        if (k_last) k_last[p] = kl;
    }
    if (nsamp) *nsamp = total;
    return 0;
}

/* Reverse mode (vector-Jacobian product) of oracle_render with respect to the TF values          */
/* (R,G,B,tau at each knot), the voxel intensities through the TF lookup, and (nullable outputs)  */
/* the feature values: dL_dg [3][N], dL_dkap [N], dL_dves [N] and dL_dgmax [1].                   */
/* dout [npix][4] = dL/d(out).  Every sample of a ray is stored, then swept back to front with    */
/* the plain adjoints of C += T a c and T' = T exp(-x); x = tau M delta with M = m w u gives      */
/* dL/dM = dL/dx tau delta, and the chain rule through m (|g| / gmax, inactive where clamped at 1),*/
/* w (|k| / (|k| + k0), derivative 0 at k = 0) and u (1 + lambda_v V).  All outputs overwritten.   */
/* near_knot (nullable, [N] bytes, test support): set to 1 at the 8 corners of every sample whose  */
/* intensity lies within knot_eps of a TF knot (the TF slope jumps there, so a lower-precision     */
/* evaluation may take the neighbouring segment), 0 elsewhere.  knot_weighted != 0: set at corner  */
/* c only if the sample lies within w_c knot_eps of a knot (w_c its trilinear weight): exactly the */
/* voxels whose change by +-knot_eps can move some sample across a knot (a kink of the loss).      */
int oracle_render_vjp(const double *I, const double *g, const double *kap, const double *ves,
                      int nx, int ny, int nz, double hx, double hy, double hz, double gmax,
                      int K, const double *knots, const double *rgba, const double *prm,
                      const double *cams, int ncam, const int32_t *pix, int64_t npix,
                      const double *dout, double *dL_dtf, double *dL_dI,
                      double *dL_dg, double *dL_dkap, double *dL_dves, double *dL_dgmax,
                      double knot_eps, int knot_weighted, uint8_t *near_knot)
{
    if (nx < 2 || ny < 2 || nz < 2 || K < 2) return -1;
    scene_t sc;
    scene_init(&sc, I, g, kap, ves, nx, ny, nz, hx, hy, hz, gmax, K, knots, rgba, prm);
    const int64_t N = (int64_t)nx * ny * nz;
    for (int e = 0; e < 4 * K; ++e) dL_dtf[e] = 0.0;
    if (dL_dI) for (int64_t v = 0; v < N; ++v) dL_dI[v] = 0.0;
    if (dL_dg) for (int64_t v = 0; v < 3 * N; ++v) dL_dg[v] = 0.0;
    if (dL_dkap) for (int64_t v = 0; v < N; ++v) dL_dkap[v] = 0.0;
    if (dL_dves) for (int64_t v = 0; v < N; ++v) dL_dves[v] = 0.0;
    if (near_knot) for (int64_t v = 0; v < N; ++v) near_knot[v] = 0;
    double gmax_acc = 0.0;
    const int want_feat = dL_dg || dL_dkap || dL_dves || dL_dgmax;
    int err = 0;
#pragma omp parallel reduction(+ : gmax_acc)
    {
        double *tfacc = (double *)calloc(4 * K, sizeof(double));
        int64_t cap = 0;
        samp_t *buf = NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            const int cid = pix[3 * p];
            double o[3], d[3], tn, tf, px[4], Tl;
            int32_t kl;
            if (!(cid >= 0 && cid < ncam && make_ray(&sc, cams + 16 * cid, pix[3 * p + 1], pix[3 * p + 2], o, d, &tn, &tf)))
                continue;
            const double delta = sc.step * fmin(hx, fmin(hy, hz));
            int64_t need = (int64_t)ceil((tf - tn) / delta) + 1;
            if (need > cap) { free(buf); cap = need; buf = (samp_t *)malloc(sizeof(samp_t) * cap); }
            if (!buf) { err = -2; continue; }
            int64_t ns = march(&sc, o, d, tn, tf, buf, cap, px, &Tl, &kl, 1);
            const double gC[3] = {dout[4 * p], dout[4 * p + 1], dout[4 * p + 2]}, gA = dout[4 * p + 3];
            double Tbar = -gA; /* A = 1 - T_end */
            for (int64_t k = ns - 1; k >= 0; --k) {
                const samp_t *s = &buf[k];
                const double e = exp(-s->x);
                const double Tnext = s->T * e;
                double dot = gC[0] * s->c[0] + gC[1] * s->c[1] + gC[2] * s->c[2];
                /* C += T a c:  a = 1 - exp(-x)  ->  da/dx = exp(-x);   T' = T exp(-x) */
                const double xbar = dot * s->T * e - Tbar * Tnext;
                double vbar[4];
                for (int ch = 0; ch < 3; ++ch) vbar[ch] = gC[ch] * s->T * s->alpha;
                vbar[3] = xbar * s->M * s->dk;
                Tbar = dot * s->alpha + Tbar * e;
                /* TF values are linear in the knot values */
                if (s->seg < 0) {
                    for (int ch = 0; ch < 4; ++ch) tfacc[ch] += vbar[ch];
                } else if (s->seg >= K - 1) {
                    for (int ch = 0; ch < 4; ++ch) tfacc[4 * (K - 1) + ch] += vbar[ch];
                } else {
                    for (int ch = 0; ch < 4; ++ch) {
                        tfacc[4 * s->seg + ch] += (1.0 - s->t) * vbar[ch];
                        tfacc[4 * (s->seg + 1) + ch] += s->t * vbar[ch];
                    }
                }
                if (near_knot) {
                    double I = 0.0;
                    for (int c8 = 0; c8 < 8; ++c8) I += s->cn.w[c8] * sc.I[s->cn.idx[c8]];
                    double dmin = INFINITY;
                    for (int kk = 0; kk < K; ++kk) dmin = fmin(dmin, fabs(I - knots[kk]));
                    for (int c8 = 0; c8 < 8; ++c8) {
                        /* weighted: a small margin covers the rounding of I (FP64) */
                        const int near = knot_weighted ? (dmin <= knot_eps * s->cn.w[c8] * (1.0 + 1e-9) + 1e-14)
                                                       : (dmin < knot_eps);
                        if (near) {
#pragma omp atomic write
                            near_knot[s->cn.idx[c8]] = 1;
                        }
                    }
                }
                if (want_feat) {
                    /* x = tau M dk */
                    const double Mbar = xbar * s->v[3] * s->dk;
                    double gvb[3] = {0.0, 0.0, 0.0}, gmb = 0.0;
                    if (sc.gmax > 0.0 && s->gn > 0.0 && s->gn < sc.gmax) {
                        const double mb = Mbar * s->w * s->u;
                        for (int a = 0; a < 3; ++a) gvb[a] = mb * sc.lg * s->gv[a] / (s->gn * sc.gmax);
                        gmb = -mb * sc.lg * s->gn / (sc.gmax * sc.gmax);
                    }
                    const double ak = fabs(s->kap);
                    const double sg = s->kap > 0.0 ? 1.0 : (s->kap < 0.0 ? -1.0 : 0.0);
                    const double kb = Mbar * s->m * s->u * sc.lk * sc.k0 * sg / ((ak + sc.k0) * (ak + sc.k0));
                    const double vb = Mbar * s->m * s->w * sc.lv;
                    gmax_acc += gmb;
                    for (int c8 = 0; c8 < 8; ++c8) {
                        const int64_t v = s->cn.idx[c8];
                        const double wc = s->cn.w[c8];
                        if (dL_dg)
                            for (int a = 0; a < 3; ++a) {
#pragma omp atomic
                                dL_dg[a * N + v] += wc * gvb[a];
                            }
                        if (dL_dkap) {
#pragma omp atomic
                            dL_dkap[v] += wc * kb;
                        }
                        if (dL_dves) {
#pragma omp atomic
                            dL_dves[v] += wc * vb;
                        }
                    }
                }
                if (dL_dI) {
                    double Ibar = 0.0;
                    for (int ch = 0; ch < 4; ++ch) Ibar += vbar[ch] * s->dv[ch];
                    if (Ibar != 0.0)
                        for (int c8 = 0; c8 < 8; ++c8) {
#pragma omp atomic
                            dL_dI[s->cn.idx[c8]] += s->cn.w[c8] * Ibar;
                        }
                }
            }
        }
#pragma omp critical
        for (int e = 0; e < 4 * K; ++e) dL_dtf[e] += tfacc[e];
        free(tfacc);
        free(buf);
    }
    if (dL_dgmax) *dL_dgmax = gmax_acc;
    return err;
}
