/*
 * Plain FP64 CPU oracle for the equivalent-charge ("replacement") fast
 * multipole method of Y. Kajima, "Notes on the Fast Multipole Method"
 * (arXiv:2212.13080).  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg are its only users.  It shares
 * no code with the GPU library.  See oracle.h for conventions.
 *
 * Parity status of each function (what pins it, see tests/test_oracle_*.py):
 *   orc_nodes / orc_lagrange   : Eq. (2) identity, Kronecker property.
 *   orc_shift_1d / _3d         : invariance property Eq. (9), Eq. (11).
 *   orc_replace                : n = 2 equals trilinear cloud-in-cell weights;
 *                                moment reproduction (Eq. (2) per axis).
 *   orc_bilinear (+ replace)   : Table 2 (E1, E2), Appendix A.1.
 *   orc_direct                 : two- and three-charge closed forms.
 *   orc_ewald                  : Madelung constant of rock salt; shape term
 *                                of cubic image sums.
 *   orc_periodic_root          : independent of the splitting parameter.
 *   orc_fmm                    : orc_fmm_pairwise at small N; Table 1 error
 *                                magnitudes vs orc_direct; symmetry; split
 *                                counts vs Sec. 3.2; continuity; exact dE/dq.
 *   orc_fmm_pairwise           : direct sum when every pair is near field;
 *                                exact 1/r for charges sitting on nodes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- basics */

void orc_nodes(int n, double sigma, double *t)
{
    /* n equally spaced points including both end points (Sec. 2.1.2),
     * optionally shrunk about the centre (Sec. 4.1). */
    if (sigma <= 0.0) sigma = 1.0;
    for (int a = 0; a < n; ++a) t[a] = sigma * ((double)a / (double)(n - 1) - 0.5) + 0.5;
}

void orc_lagrange(int n, const double *a, double x, double *g, double *dg)
{
    /* g_i(x) = prod_{k != i} (x - a_k) / prod_{k != i} (a_i - a_k)  (Sec. 2.1.1) */
    for (int i = 0; i < n; ++i) {
        double num = 1.0, den = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != i) { num *= x - a[k]; den *= a[i] - a[k]; }
        if (g) g[i] = num / den;
        if (dg) {
            double s = 0.0;
            for (int m = 0; m < n; ++m) {
                if (m == i) continue;
                double p = 1.0;
                for (int k = 0; k < n; ++k)
                    if (k != i && k != m) p *= x - a[k];
                s += p;
            }
            dg[i] = s / den;
        }
    }
}

void orc_shift_1d(int n, const double *a, const double *at, double *G)
{
    /* (j, i) entry of the shift matrix is gt_j(a_i)  (Sec. 2.1.6) */
    double g[64];
    for (int i = 0; i < n; ++i) {
        orc_lagrange(n, at, a[i], g, NULL);
        for (int j = 0; j < n; ++j) G[j * n + i] = g[j];
    }
}

void orc_replace(int n, double sigma, const double *lo, double side, int m,
                 const double *pos, const double *q, double *phi)
{
    /* Rpl_{C_n}: sum_l q_l g_i(x_l) g_j(y_l) g_k(z_l)  (Eq. (6)); the nodes of
     * the cube are lo + side * t. */
    double t[64], ax[64], ay[64], az[64], gx[64], gy[64], gz[64];
    orc_nodes(n, sigma, t);
    for (int i = 0; i < n; ++i) {
        ax[i] = lo[0] + side * t[i];
        ay[i] = lo[1] + side * t[i];
        az[i] = lo[2] + side * t[i];
    }
    memset(phi, 0, sizeof(double) * n * n * n);
    for (int l = 0; l < m; ++l) {
        orc_lagrange(n, ax, pos[3 * l + 0], gx, NULL);
        orc_lagrange(n, ay, pos[3 * l + 1], gy, NULL);
        orc_lagrange(n, az, pos[3 * l + 2], gz, NULL);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    phi[i + n * j + n * n * k] += q[l] * gx[i] * gy[j] * gz[k];
    }
}

void orc_shift_3d(int n, const double *Gx, const double *Gy, const double *Gz,
                  const double *in, double *out)
{
    /* Eq. (10): shift along x, then y, then z. */
    int n3 = n * n * n;
    double *t1 = (double *)calloc(n3, sizeof(double));
    double *t2 = (double *)calloc(n3, sizeof(double));
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int ii = 0; ii < n; ++ii) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += Gx[ii * n + i] * in[i + n * j + n * n * k];
                t1[ii + n * j + n * n * k] = s;
            }
    for (int k = 0; k < n; ++k)
        for (int jj = 0; jj < n; ++jj)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += Gy[jj * n + j] * t1[i + n * j + n * n * k];
                t2[i + n * jj + n * n * k] = s;
            }
    for (int kk = 0; kk < n; ++kk)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += Gz[kk * n + k] * t2[i + n * j + n * n * k];
                out[i + n * j + n * n * kk] = s;
            }
    free(t1);
    free(t2);
}

double orc_bilinear(int n, double sigma, const double *lo1, double s1,
                    const double *lo2, double s2, const double *v, const double *w)
{
    /* B^n_{C,C~}(v,w) = sum_a sum_b v_a w_b F(P(a), P~(b))  (Eq. (14)) */
    double t[64];
    orc_nodes(n, sigma, t);
    double acc = 0.0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double pa[3] = {lo1[0] + s1 * t[i], lo1[1] + s1 * t[j], lo1[2] + s1 * t[k]};
                double va = v[i + n * j + n * n * k];
                for (int kk = 0; kk < n; ++kk)
                    for (int jj = 0; jj < n; ++jj)
                        for (int ii = 0; ii < n; ++ii) {
                            double dx = pa[0] - (lo2[0] + s2 * t[ii]);
                            double dy = pa[1] - (lo2[1] + s2 * t[jj]);
                            double dz = pa[2] - (lo2[2] + s2 * t[kk]);
                            acc += va * w[ii + n * jj + n * n * kk] / sqrt(dx * dx + dy * dy + dz * dz);
                        }
            }
    return acc;
}

void orc_bilinear_matrix(int n, double sigma, const double *lo1, double s1,
                         const double *lo2, double s2, double *K)
{
    /* Matrix of Eq. (14): K[a*n^3 + b] = F(P(a), P~(b)). */
    double t[64];
    orc_nodes(n, sigma, t);
    int n3 = n * n * n;
    for (int a = 0; a < n3; ++a)
        for (int b = 0; b < n3; ++b) {
            double dx = (lo1[0] + s1 * t[a % n]) - (lo2[0] + s2 * t[b % n]);
            double dy = (lo1[1] + s1 * t[(a / n) % n]) - (lo2[1] + s2 * t[(b / n) % n]);
            double dz = (lo1[2] + s1 * t[a / (n * n)]) - (lo2[2] + s2 * t[b / (n * n)]);
            K[a * n3 + b] = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        }
}

/* ------------------------------------------------------------ reference sums */

int orc_direct(int N, const double *pos, const double *q, int ntarget, const int *targets,
               double *phi, double *field)
{
    /* phi_i = sum_{j != i} q_j / |x_i - x_j|, field_i = -grad phi_i */
    int nt = targets ? ntarget : N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < nt; ++t) {
        int i = targets ? targets[t] : t;
        double p = 0.0, f[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            p += q[j] / r;
            for (int a = 0; a < 3; ++a) f[a] += q[j] * d[a] / (r2 * r);
        }
        if (phi) phi[t] = p;
        if (field) for (int a = 0; a < 3; ++a) field[3 * t + a] = f[a];
    }
    return ORC_OK;
}

static int check_neutral(int N, const double *q)
{
    double s = 0.0, sa = 0.0;
    for (int i = 0; i < N; ++i) { s += q[i]; sa += fabs(q[i]); }
    return fabs(s) <= 1e-10 * sa ? ORC_OK : ORC_ENEUTRAL;
}

int orc_ewald(int N, const double *pos, const double *q, const double *origin, double box,
              double alpha, int nreal, int nrecip, int ntarget, const int *targets,
              double *phi, double *field)
{
    /* Tin-foil Ewald sum (textbook):
     *   phi_i = sum_j sum_m' q_j erfc(alpha r)/r
     *         + (4 pi / V) sum_{k != 0} exp(-k^2/4alpha^2)/k^2 Re[e^{ik.x_i} S(k)^*]
     *         - 2 alpha q_i / sqrt(pi) - pi/(alpha^2 V) sum_j q_j,
     *   S(k) = sum_j q_j e^{ik.x_j}; the k = 0 term is omitted. */
    (void)origin;
    if (check_neutral(N, q) != ORC_OK) return ORC_ENEUTRAL;
    int nt = targets ? ntarget : N;
    double V = box * box * box;
    double qsum = 0.0;
    for (int j = 0; j < N; ++j) qsum += q[j];
    int K = nrecip, nk1 = 2 * K + 1;
    int nk = nk1 * nk1 * nk1;
    double *Sre = (double *)calloc(nk, sizeof(double));
    double *Sim = (double *)calloc(nk, sizeof(double));
    if (!Sre || !Sim) { free(Sre); free(Sim); return ORC_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 8)
    for (int kk = 0; kk < nk; ++kk) {
        int nx = kk % nk1 - K, ny = (kk / nk1) % nk1 - K, nz = kk / (nk1 * nk1) - K;
        if (nx == 0 && ny == 0 && nz == 0) continue;
        double kx = 2 * PI * nx / box, ky = 2 * PI * ny / box, kz = 2 * PI * nz / box;
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < N; ++j) {
            double ph = kx * pos[3 * j] + ky * pos[3 * j + 1] + kz * pos[3 * j + 2];
            sr += q[j] * cos(ph);
            si += q[j] * sin(ph);
        }
        Sre[kk] = sr;
        Sim[kk] = si;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < nt; ++t) {
        int i = targets ? targets[t] : t;
        double p = 0.0, f[3] = {0.0, 0.0, 0.0};
        /* real space */
        for (int j = 0; j < N; ++j) {
            double d0[3];
            for (int a = 0; a < 3; ++a) {
                d0[a] = pos[3 * i + a] - pos[3 * j + a];
                d0[a] -= box * nearbyint(d0[a] / box);
            }
            for (int mz = -nreal; mz <= nreal; ++mz)
                for (int my = -nreal; my <= nreal; ++my)
                    for (int mx = -nreal; mx <= nreal; ++mx) {
                        if (j == i && mx == 0 && my == 0 && mz == 0) continue;
                        double d[3] = {d0[0] + mx * box, d0[1] + my * box, d0[2] + mz * box};
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        double r = sqrt(r2);
                        double ec = erfc(alpha * r);
                        p += q[j] * ec / r;
                        double fr = q[j] * (ec / r + 2.0 * alpha / sqrt(PI) * exp(-alpha * alpha * r2)) / r2;
                        for (int a = 0; a < 3; ++a) f[a] += fr * d[a];
                    }
        }
        /* reciprocal space */
        for (int kk = 0; kk < nk; ++kk) {
            int nx = kk % nk1 - K, ny = (kk / nk1) % nk1 - K, nz = kk / (nk1 * nk1) - K;
            if (nx == 0 && ny == 0 && nz == 0) continue;
            double kx = 2 * PI * nx / box, ky = 2 * PI * ny / box, kz = 2 * PI * nz / box;
            double k2 = kx * kx + ky * ky + kz * kz;
            double A = 4.0 * PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
            double ph = kx * pos[3 * i] + ky * pos[3 * i + 1] + kz * pos[3 * i + 2];
            double c = cos(ph), s = sin(ph);
            p += A * (c * Sre[kk] + s * Sim[kk]);
            double g = A * (s * Sre[kk] - c * Sim[kk]);
            f[0] += g * kx;
            f[1] += g * ky;
            f[2] += g * kz;
        }
        p -= 2.0 * alpha / sqrt(PI) * q[i];
        p -= PI / (alpha * alpha * V) * qsum;
        if (phi) phi[t] = p;
        if (field) for (int a = 0; a < 3; ++a) field[3 * t + a] = f[a];
    }
    free(Sre);
    free(Sim);
    return ORC_OK;
}

/* Ewald Green's function at unit box side minus the 27 nearest images:
 * the interaction of a unit charge at 0 with the far images (|m|_inf >= 2)
 * of a unit charge at r, in the tin-foil convention. */
static double far_image_green(const double r[3], double alpha)
{
    const int R = 4, K = 8;
    double s = 0.0;
    for (int mz = -R; mz <= R; ++mz)
        for (int my = -R; my <= R; ++my)
            for (int mx = -R; mx <= R; ++mx) {
                double d[3] = {r[0] + mx, r[1] + my, r[2] + mz};
                double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                int near = abs(mx) <= 1 && abs(my) <= 1 && abs(mz) <= 1;
                if (near)  /* erfc(a rho)/rho - 1/rho = -erf(a rho)/rho */
                    s += rho > 0.0 ? -erf(alpha * rho) / rho : -2.0 * alpha / sqrt(PI);
                else
                    s += erfc(alpha * rho) / rho;
            }
    for (int nz = -K; nz <= K; ++nz)
        for (int ny = -K; ny <= K; ++ny)
            for (int nx = -K; nx <= K; ++nx) {
                if (nx == 0 && ny == 0 && nz == 0) continue;
                double k[3] = {2 * PI * nx, 2 * PI * ny, 2 * PI * nz};
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                s += 4.0 * PI * exp(-k2 / (4.0 * alpha * alpha)) / k2 *
                     cos(k[0] * r[0] + k[1] * r[1] + k[2] * r[2]);
            }
    return s - PI / (alpha * alpha);
}

int orc_periodic_root_alpha(int n, double sigma, double alpha, double *T)
{
    double t[64];
    orc_nodes(n, sigma, t);
    int n3 = n * n * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int a = 0; a < n3; ++a) {
        double xa[3] = {t[a % n], t[(a / n) % n], t[a / (n * n)]};
        for (int b = 0; b < n3; ++b) {
            double xb[3] = {t[b % n], t[(b / n) % n], t[b / (n * n)]};
            double r[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
            T[a * n3 + b] = far_image_green(r, alpha);
        }
    }
    return ORC_OK;
}

int orc_periodic_root(int n, double sigma, double *T)
{
    return orc_periodic_root_alpha(n, sigma, 2.0, T);
}

/* ------------------------------------------------------------------ split */

typedef struct {
    int cell[3];     /* leaf cell (integer coordinates, in range)       */
    double u[3];     /* coordinates local to that leaf, in [0, 1]       */
    double x[3];     /* position relative to the box origin (folded)    */
    double Q;        /* q * w                                           */
    double w;        /* split weight                                    */
    double dw[3];    /* d w / d x_a                                     */
    int parent;      /* index of the original charge                    */
} frag_t;

typedef struct {
    int n;
    int cell[16];
    double u[16], x[16], om[16], dom[16];
} axis_pieces_t;

static int is_periodic(int b) { return b == ORC_PERIODIC || b == ORC_PERIODIC_CONTINUOUS; }
static int is_continuous(int b) { return b == ORC_FREE_CONTINUOUS || b == ORC_PERIODIC_CONTINUOUS; }

static double default_d(const orc_params *p)
{
    double s = p->box / (double)(1 << p->levels);
    return p->split_d > 0.0 ? p->split_d : s / 256.0;
}

/* Pieces of one axis: one unsplit piece, or the n-division points of the
 * segment of length 2d centred on the nearby face (Sec. 2.3).  A point on
 * the face (odd n) is halved into both cells; in periodic modes pieces
 * beyond a wall are folded back by the box side (Sec. 4.2). */
static void axis_split(const orc_params *p, double xr, axis_pieces_t *ap)
{
    int n = p->order, D = 1 << p->levels;
    double h = p->box, s = h / (double)D, d = default_d(p);
    int c = (int)floor(xr / s);
    if (c >= D) c = D - 1;
    if (c < 0) c = 0;
    double dlo = xr - c * s, dhi = (c + 1) * s - xr;
    int per = is_periodic(p->boundary);
    int fb = -1;
    if (is_continuous(p->boundary)) {
        if (dlo < d && (per || c > 0)) fb = c;
        else if (dhi < d && (per || c < D - 1)) fb = c + 1;
    }
    if (fb < 0) {
        ap->n = 1;
        ap->cell[0] = c;
        ap->u[0] = xr / s - c;
        ap->x[0] = xr;
        ap->om[0] = 1.0;
        ap->dom[0] = 0.0;
        return;
    }
    double b = fb * s;
    double tau = (xr - (b - d)) / (2.0 * d);
    double tn[16], g[16], dg[16];
    orc_nodes(n, 1.0, tn);
    orc_lagrange(n, tn, tau, g, dg);
    int m = 0;
    for (int k = 0; k < n; ++k) {
        double pk = b - d + 2.0 * d * k / (double)(n - 1);
        int sides[2], ns = 0;
        double frac = 1.0;
        if (2 * k < n - 1) sides[ns++] = 0;
        else if (2 * k > n - 1) sides[ns++] = 1;
        else { sides[ns++] = 0; sides[ns++] = 1; frac = 0.5; pk = b; }
        for (int e = 0; e < ns; ++e) {
            int cell = sides[e] == 0 ? fb - 1 : fb;
            double xx = pk;
            if (cell < 0) { cell += D; xx += h; }
            if (cell >= D) { cell -= D; xx -= h; }
            ap->cell[m] = cell;
            ap->x[m] = xx;
            ap->u[m] = xx / s - cell;
            ap->om[m] = frac * g[k];
            ap->dom[m] = frac * dg[k] / (2.0 * d);
            ++m;
        }
    }
    ap->n = m;
}

/* Wrap (periodic) or check (free) one coordinate relative to the origin. */
static int box_coord(const orc_params *p, double x, double o, double *xr)
{
    double h = p->box, v = x - o;
    if (!isfinite(v)) return ORC_ENONFINITE;
    if (is_periodic(p->boundary)) {
        v -= h * floor(v / h);
        if (v >= h) v -= h;
        if (v < 0.0) v = 0.0;
    } else if (v < 0.0 || v > h) {
        return ORC_EBOX;
    }
    *xr = v;
    return ORC_OK;
}

static int make_fragments(const orc_params *p, int N, const double *pos, const double *q,
                          frag_t **out, int *nfrag, int *split_mask, int *nsplit)
{
    int cap = N + 1024, nf = 0, ns = 0;
    frag_t *f = (frag_t *)malloc(sizeof(frag_t) * cap);
    if (!f) return ORC_ENOMEM;
    for (int i = 0; i < N; ++i) {
        axis_pieces_t ap[3];
        int mask = 0;
        for (int a = 0; a < 3; ++a) {
            double xr;
            int rc = box_coord(p, pos[3 * i + a], p->origin[a], &xr);
            if (rc == ORC_OK && !isfinite(q[i])) rc = ORC_ENONFINITE;
            if (rc != ORC_OK) { free(f); return rc; }
            axis_split(p, xr, &ap[a]);
            if (ap[a].n > 1) mask |= 1 << a;
        }
        if (split_mask) split_mask[i] = mask;
        if (mask) ++ns;
        int cnt = ap[0].n * ap[1].n * ap[2].n;
        if (nf + cnt > cap) {
            cap = 2 * cap + cnt;
            frag_t *g = (frag_t *)realloc(f, sizeof(frag_t) * cap);
            if (!g) { free(f); return ORC_ENOMEM; }
            f = g;
        }
        for (int kz = 0; kz < ap[2].n; ++kz)
            for (int ky = 0; ky < ap[1].n; ++ky)
                for (int kx = 0; kx < ap[0].n; ++kx) {
                    frag_t *r = &f[nf++];
                    int k[3] = {kx, ky, kz};
                    double om[3], dom[3];
                    for (int a = 0; a < 3; ++a) {
                        r->cell[a] = ap[a].cell[k[a]];
                        r->u[a] = ap[a].u[k[a]];
                        r->x[a] = ap[a].x[k[a]];
                        om[a] = ap[a].om[k[a]];
                        dom[a] = ap[a].dom[k[a]];
                    }
                    r->w = om[0] * om[1] * om[2];
                    r->dw[0] = dom[0] * om[1] * om[2];
                    r->dw[1] = om[0] * dom[1] * om[2];
                    r->dw[2] = om[0] * om[1] * dom[2];
                    r->Q = q[i] * r->w;
                    r->parent = i;
                }
    }
    *out = f;
    *nfrag = nf;
    if (nsplit) *nsplit = ns;
    return ORC_OK;
}

static int validate(const orc_params *p)
{
    if (!p || p->levels < 2 || p->levels > 10 || p->order < 2 || p->order > 12 || !(p->box > 0.0))
        return ORC_EINVAL;
    if (p->boundary < 0 || p->boundary > 3) return ORC_EINVAL;
    double s = p->box / (double)(1 << p->levels);
    double d = default_d(p);
    if (!(d > 0.0) || !(2.0 * d < s)) return ORC_EINVAL;
    return ORC_OK;
}

int orc_split_count(const orc_params *p, int N, const double *pos, int *nsplit, int *nfrag)
{
    int rc = validate(p);
    if (rc) return rc;
    double *q = (double *)malloc(sizeof(double) * (N > 0 ? N : 1));
    for (int i = 0; i < N; ++i) q[i] = 1.0;
    frag_t *f = NULL;
    rc = make_fragments(p, N, pos, q, &f, nfrag, NULL, nsplit);
    free(q);
    free(f);
    return rc;
}

/* ------------------------------------------------------------------- FMM */

static long cells_at(int l) { return 1L << (3 * l); }
static long level_offset(int l) { long o = 0; for (int k = 0; k < l; ++k) o += cells_at(k); return o; }

int orc_fmm(const orc_params *p, int N, const double *pos, const double *q,
            double *phi_out, double *field_out, double *field_paper, double *energy,
            double *phi_levels, double *L_levels)
{
    int rc = validate(p);
    if (rc) return rc;
    const int n = p->order, n3 = n * n * n, Lf = p->levels;
    const int per = is_periodic(p->boundary);
    const double h = p->box;
    const double sigma = p->node_shrink > 0.0 ? p->node_shrink : 1.0;
    if (per && check_neutral(N, q) != ORC_OK) return ORC_ENEUTRAL;

    /* Split (Sec. 2.3, Sec. 4.2), then the charge set is the fragment set. */
    frag_t *fr = NULL;
    int nf = 0;
    int *mask = (int *)calloc(N > 0 ? N : 1, sizeof(int));
    rc = make_fragments(p, N, pos, q, &fr, &nf, mask, NULL);
    if (rc) { free(mask); return rc; }

    /* Step 1: divide the box; list the fragments of every finest cell. */
    const int D = 1 << Lf;
    const long nleaf = cells_at(Lf);
    int *start = (int *)calloc((size_t)(nleaf > 0 ? nleaf + 1 : 1), sizeof(int));
    int *order = (int *)malloc(sizeof(int) * (nf > 0 ? nf : 1));
    for (int m = 0; m < nf; ++m) {
        long c = fr[m].cell[0] + (long)D * (fr[m].cell[1] + (long)D * fr[m].cell[2]);
        start[c + 1]++;
    }
    for (long c = 0; c < nleaf; ++c) start[c + 1] += start[c];
    {
        int *fill = (int *)calloc((size_t)(nleaf > 0 ? nleaf : 1), sizeof(int));
        for (int m = 0; m < nf; ++m) {
            long c = fr[m].cell[0] + (long)D * (fr[m].cell[1] + (long)D * fr[m].cell[2]);
            order[start[c] + fill[c]++] = m;
        }
        free(fill);
    }

    /* Unit-cell nodes, child->parent shift matrices G_b (b = child half),
     * and their transposes for the downward pass. */
    double t[64];
    orc_nodes(n, sigma, t);
    double G[2][144], Gt[2][144];
    for (int b = 0; b < 2; ++b) {
        double a[64];
        for (int i = 0; i < n; ++i) a[i] = 0.5 * (b + t[i]);  /* child nodes in parent units */
        orc_shift_1d(n, a, t, G[b]);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) Gt[b][i * n + j] = G[b][j * n + i];
    }

    const long total = level_offset(Lf + 1);
    double *Phi = (double *)calloc((size_t)total * n3, sizeof(double));
    double *Lv = (double *)calloc((size_t)total * n3, sizeof(double));
    if (!Phi || !Lv || !start || !order) {
        free(Phi); free(Lv); free(start); free(order); free(fr); free(mask);
        return ORC_ENOMEM;
    }

    /* Step 2: upward pass.  Replace at the finest cells (Eq. (6)) ... */
    {
        double *PhiL = Phi + (size_t)level_offset(Lf) * n3;
#pragma omp parallel for schedule(dynamic, 64)
        for (long c = 0; c < nleaf; ++c) {
            double gx[64], gy[64], gz[64];
            double *ph = PhiL + (size_t)c * n3;
            for (int e = start[c]; e < start[c + 1]; ++e) {
                const frag_t *f = &fr[order[e]];
                orc_lagrange(n, t, f->u[0], gx, NULL);
                orc_lagrange(n, t, f->u[1], gy, NULL);
                orc_lagrange(n, t, f->u[2], gz, NULL);
                for (int k = 0; k < n; ++k)
                    for (int j = 0; j < n; ++j)
                        for (int i = 0; i < n; ++i)
                            ph[i + n * j + n * n * k] += f->Q * gx[i] * gy[j] * gz[k];
            }
        }
    }
    /* ... then shift the eight children to their parent and add (Eq. (10)). */
    for (int l = Lf; l >= 1; --l) {
        const int Dl = 1 << l, Dp = Dl >> 1;
        double *Pc = Phi + (size_t)level_offset(l) * n3;
        double *Pp = Phi + (size_t)level_offset(l - 1) * n3;
#pragma omp parallel for schedule(static)
        for (long P = 0; P < cells_at(l - 1); ++P) {
            int X = P % Dp, Y = (P / Dp) % Dp, Z = P / ((long)Dp * Dp);
            double *tmp = (double *)malloc(sizeof(double) * n3);
            for (int bz = 0; bz < 2; ++bz)
                for (int by = 0; by < 2; ++by)
                    for (int bx = 0; bx < 2; ++bx) {
                        long c = (2 * X + bx) + (long)Dl * ((2 * Y + by) + (long)Dl * (2 * Z + bz));
                        orc_shift_3d(n, G[bx], G[by], G[bz], Pc + (size_t)c * n3, tmp);
                        for (int a = 0; a < n3; ++a) Pp[(size_t)P * n3 + a] += tmp[a];
                    }
            free(tmp);
        }
    }

    /* Step 3: downward pass.  Psi_C(v) = L_C . v.  Psi vanishes at levels 0
     * and 1 in free space; the periodic modes start from the far images of
     * the whole box at level 0. */
    if (per) {
        double *T = (double *)malloc(sizeof(double) * n3 * n3);
        orc_periodic_root(n, sigma, T);
        for (int a = 0; a < n3; ++a) {
            double s = 0.0;
            for (int b = 0; b < n3; ++b) s += T[a * n3 + b] * Phi[b];
            Lv[a] = s / h;
        }
        free(T);
    }
    /* Coulomb matrices of the 7^3 displacements between same-level cells,
     * in units of the cell side: F(P(a), P~(b)) * side = 1/|t_a - t_b - o|. */
    double *K = (double *)malloc(sizeof(double) * 343 * n3 * n3);
    for (int oi = 0; oi < 343; ++oi) {
        int ox = oi % 7 - 3, oy = (oi / 7) % 7 - 3, oz = oi / 49 - 3;
        if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
        for (int a = 0; a < n3; ++a)
            for (int b = 0; b < n3; ++b) {
                double dx = t[a % n] - t[b % n] - ox;
                double dy = t[(a / n) % n] - t[(b / n) % n] - oy;
                double dz = t[a / (n * n)] - t[b / (n * n)] - oz;
                K[(size_t)oi * n3 * n3 + a * n3 + b] = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
            }
    }
    for (int l = 1; l <= Lf; ++l) {
        const int Dl = 1 << l, Dp = Dl >> 1;
        const double inv_side = (double)Dl / h;
        double *Lc = Lv + (size_t)level_offset(l) * n3;
        double *Lp = Lv + (size_t)level_offset(l - 1) * n3;
        double *Pl = Phi + (size_t)level_offset(l) * n3;
        const int interact = per || l >= 2;
#pragma omp parallel for schedule(dynamic, 16)
        for (long c = 0; c < cells_at(l); ++c) {
            int x = c % Dl, y = (c / Dl) % Dl, z = c / ((long)Dl * Dl);
            long P = (x >> 1) + (long)Dp * ((y >> 1) + (long)Dp * (z >> 1));
            double *Lcc = Lc + (size_t)c * n3;
            /* Psi_child = Psi_parent o shift_{child -> parent} */
            orc_shift_3d(n, Gt[x & 1], Gt[y & 1], Gt[z & 1], Lp + (size_t)P * n3, Lcc);
            if (!interact) continue;
            /* interaction list: children of the parent's neighbours that are
             * not adjacent to this cell */
            for (int oz = -2 - (z & 1); oz <= 3 - (z & 1); ++oz)
                for (int oy = -2 - (y & 1); oy <= 3 - (y & 1); ++oy)
                    for (int ox = -2 - (x & 1); ox <= 3 - (x & 1); ++ox) {
                        if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
                        int sx = x + ox, sy = y + oy, sz = z + oz;
                        if (per) {
                            sx = ((sx % Dl) + Dl) % Dl;
                            sy = ((sy % Dl) + Dl) % Dl;
                            sz = ((sz % Dl) + Dl) % Dl;
                        } else if (sx < 0 || sy < 0 || sz < 0 || sx >= Dl || sy >= Dl || sz >= Dl) {
                            continue;
                        }
                        long cs = sx + (long)Dl * (sy + (long)Dl * sz);
                        int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
                        const double *Ko = K + (size_t)oi * n3 * n3;
                        const double *ps = Pl + (size_t)cs * n3;
                        for (int a = 0; a < n3; ++a) {
                            double s = 0.0;
                            for (int b = 0; b < n3; ++b) s += Ko[a * n3 + b] * ps[b];
                            Lcc[a] += inv_side * s;
                        }
                    }
        }
    }
    free(K);

    /* Step 4: far-field potential (and field) at every fragment:
     * Psi_leaf applied to the replacement of a unit charge there. */
    double *fphi = (double *)calloc(nf > 0 ? nf : 1, sizeof(double));
    double *ffld = (double *)calloc(3 * (nf > 0 ? nf : 1), sizeof(double));
    {
        const double inv_s = (double)D / h;
        double *LL = Lv + (size_t)level_offset(Lf) * n3;
#pragma omp parallel for schedule(static)
        for (int m = 0; m < nf; ++m) {
            const frag_t *f = &fr[m];
            long c = f->cell[0] + (long)D * (f->cell[1] + (long)D * f->cell[2]);
            double gx[64], gy[64], gz[64], dx[64], dy[64], dz[64];
            orc_lagrange(n, t, f->u[0], gx, dx);
            orc_lagrange(n, t, f->u[1], gy, dy);
            orc_lagrange(n, t, f->u[2], gz, dz);
            double s = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
            for (int k = 0; k < n; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        double Lval = LL[(size_t)c * n3 + i + n * j + n * n * k];
                        s += Lval * gx[i] * gy[j] * gz[k];
                        g0 += Lval * dx[i] * gy[j] * gz[k];
                        g1 += Lval * gx[i] * dy[j] * gz[k];
                        g2 += Lval * gx[i] * gy[j] * dz[k];
                    }
            fphi[m] = s;
            ffld[3 * m + 0] = -g0 * inv_s;
            ffld[3 * m + 1] = -g1 * inv_s;
            ffld[3 * m + 2] = -g2 * inv_s;
        }
    }

    /* Step 5: near field, directly over the same and the 26 adjacent finest
     * cells; fragments of the same original charge do not interact. */
#pragma omp parallel for schedule(dynamic, 64)
    for (int m = 0; m < nf; ++m) {
        const frag_t *f = &fr[m];
        double ps = 0.0, fs[3] = {0.0, 0.0, 0.0};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int ux = f->cell[0] + dx, uy = f->cell[1] + dy, uz = f->cell[2] + dz;
                    double img[3] = {0.0, 0.0, 0.0};
                    if (per) {
                        int wx = ((ux % D) + D) % D, wy = ((uy % D) + D) % D, wz = ((uz % D) + D) % D;
                        img[0] = (double)((ux - wx) / D) * h;
                        img[1] = (double)((uy - wy) / D) * h;
                        img[2] = (double)((uz - wz) / D) * h;
                        ux = wx; uy = wy; uz = wz;
                    } else if (ux < 0 || uy < 0 || uz < 0 || ux >= D || uy >= D || uz >= D) {
                        continue;
                    }
                    long c = ux + (long)D * (uy + (long)D * uz);
                    for (int e = start[c]; e < start[c + 1]; ++e) {
                        const frag_t *g = &fr[order[e]];
                        if (g->parent == f->parent) continue;
                        double d[3] = {f->x[0] - (g->x[0] + img[0]), f->x[1] - (g->x[1] + img[1]),
                                       f->x[2] - (g->x[2] + img[2])};
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        double r = sqrt(r2);
                        ps += g->Q / r;
                        for (int a = 0; a < 3; ++a) fs[a] += g->Q * d[a] / (r2 * r);
                    }
                }
        fphi[m] += ps;
        for (int a = 0; a < 3; ++a) ffld[3 * m + a] += fs[a];
    }

    /* Back to the original charges: phi_i = sum_m w_m phi(p_m) = dE/dq_i;
     * along a split axis the fragments stay put and only their weights move
     * with the charge, so the exact gradient there is the dw term. */
    double E = 0.0;
    {
        int m = 0;
        for (int i = 0; i < N; ++i) {
            double pi = 0.0, fe[3] = {0.0, 0.0, 0.0}, fp[3] = {0.0, 0.0, 0.0};
            for (; m < nf && fr[m].parent == i; ++m) {
                pi += fr[m].w * fphi[m];
                for (int a = 0; a < 3; ++a) {
                    fp[a] += fr[m].w * ffld[3 * m + a];
                    if (mask[i] & (1 << a)) fe[a] -= fr[m].dw[a] * fphi[m];
                    else fe[a] += fr[m].w * ffld[3 * m + a];
                }
            }
            if (phi_out) phi_out[i] = pi;
            if (field_out) for (int a = 0; a < 3; ++a) field_out[3 * i + a] = fe[a];
            if (field_paper) for (int a = 0; a < 3; ++a) field_paper[3 * i + a] = fp[a];
            E += 0.5 * q[i] * pi;
        }
    }
    if (energy) *energy = E;
    if (phi_levels) memcpy(phi_levels, Phi, sizeof(double) * (size_t)total * n3);
    if (L_levels) memcpy(L_levels, Lv, sizeof(double) * (size_t)total * n3);

    free(fphi); free(ffld); free(Phi); free(Lv); free(start); free(order); free(fr); free(mask);
    return ORC_OK;
}

/* ------------------------------------------------------ pairwise closed form */

static int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

int orc_fmm_pairwise(const orc_params *p, int N, const double *pos, const double *q,
                     double *phi_out, double *energy)
{
    int rc = validate(p);
    if (rc) return rc;
    const int n = p->order, n3 = n * n * n, Lf = p->levels, D = 1 << Lf;
    const int per = is_periodic(p->boundary);
    const double h = p->box;
    const double sigma = p->node_shrink > 0.0 ? p->node_shrink : 1.0;
    if (per && check_neutral(N, q) != ORC_OK) return ORC_ENEUTRAL;
    frag_t *fr = NULL;
    int nf = 0;
    rc = make_fragments(p, N, pos, q, &fr, &nf, NULL, NULL);
    if (rc) return rc;
    double *T = NULL;
    if (per) {
        T = (double *)malloc(sizeof(double) * n3 * n3);
        orc_periodic_root(n, sigma, T);
    }
    double *fphi = (double *)calloc(nf > 0 ? nf : 1, sizeof(double));
    const int R = per ? 1 : 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < nf; ++m) {
        const frag_t *f = &fr[m];
        double acc = 0.0;
        double *va = (double *)malloc(sizeof(double) * n3);
        double *vb = (double *)malloc(sizeof(double) * n3);
        for (int mp = 0; mp < nf; ++mp) {
            const frag_t *g = &fr[mp];
            for (int iz = -R; iz <= R; ++iz)
                for (int iy = -R; iy <= R; ++iy)
                    for (int ix = -R; ix <= R; ++ix) {
                        int im[3] = {ix, iy, iz};
                        int A[3], B[3];
                        for (int a = 0; a < 3; ++a) { A[a] = f->cell[a]; B[a] = g->cell[a] + im[a] * D; }
                        /* first level at which the ancestors are not adjacent */
                        int lev = -1;
                        for (int l = 0; l <= Lf && lev < 0; ++l) {
                            int sh = 1 << (Lf - l), sep = 0;
                            for (int a = 0; a < 3; ++a)
                                if (abs(floor_div(A[a], sh) - floor_div(B[a], sh)) > 1) sep = 1;
                            if (sep) lev = l;
                        }
                        double gpos[3] = {g->x[0] + im[0] * h, g->x[1] + im[1] * h, g->x[2] + im[2] * h};
                        if (lev < 0) {
                            if (g->parent == f->parent) continue;
                            double d[3] = {f->x[0] - gpos[0], f->x[1] - gpos[1], f->x[2] - gpos[2]};
                            acc += g->Q / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        } else {
                            int sh = 1 << (Lf - lev);
                            double side = h / (double)(1 << lev);
                            double loA[3], loB[3];
                            for (int a = 0; a < 3; ++a) {
                                loA[a] = floor_div(A[a], sh) * side;
                                loB[a] = floor_div(B[a], sh) * side;
                            }
                            double one = 1.0;
                            orc_replace(n, sigma, loA, side, 1, f->x, &one, va);
                            orc_replace(n, sigma, loB, side, 1, gpos, &g->Q, vb);
                            acc += orc_bilinear(n, sigma, loA, side, loB, side, va, vb);
                        }
                    }
            if (per) {
                double lo0[3] = {0.0, 0.0, 0.0}, one = 1.0;
                orc_replace(n, sigma, lo0, h, 1, f->x, &one, va);
                orc_replace(n, sigma, lo0, h, 1, g->x, &g->Q, vb);
                double s = 0.0;
                for (int a = 0; a < n3; ++a)
                    for (int b = 0; b < n3; ++b) s += va[a] * T[a * n3 + b] * vb[b];
                acc += s / h;
            }
        }
        fphi[m] = acc;
        free(va);
        free(vb);
    }
    double E = 0.0;
    int m = 0;
    for (int i = 0; i < N; ++i) {
        double pi = 0.0;
        for (; m < nf && fr[m].parent == i; ++m) pi += fr[m].w * fphi[m];
        if (phi_out) phi_out[i] = pi;
        E += 0.5 * q[i] * pi;
    }
    if (energy) *energy = E;
    free(fphi);
    free(T);
    free(fr);
    return ORC_OK;
}
