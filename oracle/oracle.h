/*
 * Plain FP64 CPU oracle for the equivalent-charge ("replacement") fast
 * multipole method of Y. Kajima, "Notes on the Fast Multipole Method"
 * (arXiv:2212.13080).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the GPU library, and it is written
 * for a reader checking it against the paper, not for speed.
 *
 * Conventions
 *   - n    : order of replacement = number of n-division points per axis
 *            (Sec. 2.1.2); a cell holds n^3 equivalent charges.
 *   - L    : finest level l_f >= 2 (Sec. 2.2, step 1).
 *   - Node index inside a cell: a = i + n*j + n*n*k  (x fastest).
 *   - Cell index at level l (D = 2^l cells per axis): c = x + D*(y + D*z).
 *   - Pair potential q q'/r, Coulomb constant 1 (Sec. 3.1).
 *   - phi[i]   : potential at charge i from every other charge (self pair
 *                excluded), so that E = 1/2 sum_i q_i phi[i].
 *   - field[i] : -grad phi at charge i; the force is q_i * field[i].
 *
 * Every function returns 0 on success or a negative code (see ORC_E*).
 */
#ifndef EQFMM_ORACLE_H
#define EQFMM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FREE = 0, ORC_FREE_CONTINUOUS = 1, ORC_PERIODIC = 2, ORC_PERIODIC_CONTINUOUS = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EBOX = -2, ORC_ENEUTRAL = -3, ORC_ENONFINITE = -4,
       ORC_ENOMEM = -5 };

typedef struct {
    int    levels;       /* finest level l_f >= 2                             */
    int    order;        /* n >= 2 points per axis                            */
    int    boundary;     /* ORC_FREE .. ORC_PERIODIC_CONTINUOUS               */
    double origin[3];    /* lower corner of the box                           */
    double box;          /* side h > 0                                        */
    double split_d;      /* split half-width d; <= 0 selects leaf side / 256  */
    double node_shrink;  /* node lattice scale sigma in (0,1]; <= 0 selects 1 */
} orc_params;

/* n-division points of the unit segment, scaled by sigma about its centre
 * (Sec. 2.1.2; reduced arrangement of Sec. 4.1 when sigma < 1). */
void orc_nodes(int n, double sigma, double *t);

/* Lagrange basis g_i(x) on the n distinct nodes a[] and its derivative
 * (Sec. 2.1.1, Eq. (1)). */
void orc_lagrange(int n, const double *a, double x, double *g, double *dg);

/* 1-D shift matrix from node set a[] to node set at[] (Sec. 2.1.6):
 * G[j*n + i] = gt_j(a_i), gt the Lagrange basis on at[]. */
void orc_shift_1d(int n, const double *a, const double *at, double *G);

/* 3-D replacement of m charges with respect to the cube [lo, lo+side]^3
 * (Sec. 2.1.5, Eq. (6)); phi has n^3 entries. */
void orc_replace(int n, double sigma, const double *lo, double side, int m,
                 const double *pos, const double *q, double *phi);

/* 3-D shift as three axis-wise 1-D shifts (Sec. 2.1.6, Eq. (10)). */
void orc_shift_3d(int n, const double *Gx, const double *Gy, const double *Gz,
                  const double *in, double *out);

/* Bilinear form B^n_{C,C~}(v, w) of Eq. (14) between cubes C=[lo1,lo1+s1]^3
 * and C~=[lo2,lo2+s2]^3. */
double orc_bilinear(int n, double sigma, const double *lo1, double s1,
                    const double *lo2, double s2, const double *v, const double *w);

/* The matrix of that bilinear form, K[a*n^3 + b] = F(P(a), P~(b)). */
void orc_bilinear_matrix(int n, double sigma, const double *lo1, double s1,
                         const double *lo2, double s2, double *K);

/* O(N^2) direct sum in free space over the listed targets (NULL = all). */
int orc_direct(int N, const double *pos, const double *q, int ntarget, const int *targets,
               double *phi, double *field);

/* Tin-foil Ewald sum of a neutral periodic system in the cube
 * [origin, origin+box)^3 over the listed targets (NULL = all). alpha is
 * the splitting parameter, real-space images |m_i| <= nreal around the
 * minimum image, reciprocal vectors |k_i| <= nrecip (units of 2 pi/box). */
int orc_ewald(int N, const double *pos, const double *q, const double *origin, double box,
              double alpha, int nreal, int nrecip, int ntarget, const int *targets,
              double *phi, double *field);

/* Split statistics (Sec. 2.3): number of charges split and number of point
 * charges after the split. */
int orc_split_count(const orc_params *p, int N, const double *pos, int *nsplit, int *nfrag);

/* The replacement FMM of Sec. 2.2 (+ Sec. 2.3 / Sec. 4.2 variants).
 * Outputs may be NULL.  field_paper is the force rule stated at the end of
 * Sec. 2.3 (sum of the fields felt by the split charges, weighted); field is
 * minus the exact gradient of the computed energy divided by q.
 * If phi_levels / L_levels are non-NULL they receive Phi and the local
 * vectors of every level, level 0 first, each level 8^l * n^3 values. */
int orc_fmm(const orc_params *p, int N, const double *pos, const double *q,
            double *phi, double *field, double *field_paper, double *energy,
            double *phi_levels, double *L_levels);

/* Pairwise closed form of the same approximation (no tree passes), for
 * small N: by the invariance property each fragment pair interacts through
 * the replacement of both at the level where their ancestors first become
 * well separated, or directly when their leaves are adjacent. */
int orc_fmm_pairwise(const orc_params *p, int N, const double *pos, const double *q,
                     double *phi, double *energy);

/* Root operator of the periodic modes: far images of the box (all images
 * outside the 3x3x3 block around it) acting on the box's own n^3 lattice,
 * built from the tin-foil Ewald Green's function; T has n^3 x n^3 entries
 * at unit box side. */
int orc_periodic_root(int n, double sigma, double *T);
int orc_periodic_root_alpha(int n, double sigma, double alpha, double *T);

#ifdef __cplusplus
}
#endif
#endif
