/*
 * eqfmm — equivalent-charge ("replacement") fast multipole method on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Y. Kajima, "Notes on the Fast Multipole Method" (arXiv:2212.13080).
 *   - replacement of the charges of a finest cell by n^3 fixed charges on the
 *     cell's n-division points (Sec. 2.1.5, Eq. (6));
 *   - shift of those charges between child and parent cells (Sec. 2.1.6,
 *     Eq. (10)) for the upward and downward passes (Sec. 2.2, steps 2-3);
 *   - far interaction of well-separated cells as the Coulomb interaction of
 *     their fixed charges, the bilinear form of Eq. (14);
 *   - near field summed directly over the same and the 26 adjacent finest
 *     cells (Sec. 1, Sec. 2.2 step 5);
 *   - the continuous variant that splits charges near finest-cell faces
 *     (Sec. 2.3) and its periodic form that also splits at the walls and
 *     folds outside pieces back into the box (Sec. 4.2).
 *
 * Problem statement (Sec. 2.2): N point charges q_i at x_i in the cube
 * [origin, origin + box)^3, pair energy q q' / r (Coulomb constant 1).
 * Outputs per charge: the potential phi_i (every other charge, self
 * excluded), the field = -grad phi_i (force = q_i * field), and the total
 * energy E = 1/2 sum_i q_i phi_i.  The periodic modes give the tin-foil
 * (conducting boundary) lattice sum of a neutral box.
 *
 * Memory ownership: the caller owns every device buffer (plan buffer,
 * workspace, inputs, outputs).  The library never allocates device memory;
 * it owns only the host-side plan object.  All device pointers are HIP
 * device addresses on the current device; `stream` is a hipStream_t (NULL =
 * default stream).  Work is enqueued on that stream (the forward calls also
 * use the plan's own stream, joined back into the caller's before the final
 * kernels).  eqfmm_forward blocks once, at its end, to read back a 4-byte
 * status; eqfmm_forward_async never blocks.
 *
 * Error behaviour: every call returns EQFMM_OK (0) or a negative code.
 * Data-dependent errors (EBOX, ENEUTRAL, ENONFINITE, fragment capacity) are
 * detected on the device; every kernel stays within its buffers whatever the
 * input (prefix sums are clamped to the fragment capacity), the outputs are
 * then unspecified, and the code is returned by eqfmm_forward or written to
 * the status word of eqfmm_forward_async.  eqfmm_strerror() names a code.
 */
#ifndef EQFMM_H
#define EQFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EQFMM_FREE = 0,                /* Sec. 2.2: free space                         */
    EQFMM_FREE_CONTINUOUS = 1,     /* Sec. 2.3: split at interior finest-cell faces */
    EQFMM_PERIODIC = 2,            /* periodic box, no split                       */
    EQFMM_PERIODIC_CONTINUOUS = 3  /* Sec. 4.2: split at every face and the walls  */
};

enum {
    EQFMM_FP64 = 0,          /* all arithmetic in double                          */
    EQFMM_FP32 = 1,          /* float arithmetic, energy reduced in double        */
    EQFMM_FP32_BF16FAR = 2   /* as FP32, far-field products with bf16 inputs and
                                float accumulation on the matrix cores            */
};

enum {
    EQFMM_OK = 0,
    EQFMM_EINVAL = -1,      /* bad parameter or NULL required pointer               */
    EQFMM_EBOX = -2,        /* free modes: a position outside [origin, origin+box]  */
    EQFMM_ENEUTRAL = -3,    /* periodic modes: |sum q| > 1e-10 * sum |q|            */
    EQFMM_ENONFINITE = -4,  /* a position or charge is NaN or infinite              */
    EQFMM_EWORKSPACE = -5,  /* workspace too small or fragment capacity exceeded    */
    EQFMM_EHIP = -6,        /* a HIP runtime call failed                            */
    EQFMM_ESTATE = -7       /* backward without a matching forward on this workspace,
                               or forward before eqfmm_plan_upload                    */
};

typedef struct {
    int32_t levels;          /* finest level l_f, 2 <= l_f <= 8 (Sec. 2.2 step 1)        */
    int32_t order;           /* n = points per axis, 2 <= n <= 7 (Sec. 2.1.2)            */
    int32_t boundary;        /* EQFMM_FREE ... EQFMM_PERIODIC_CONTINUOUS                 */
    int32_t precision;       /* EQFMM_FP64, EQFMM_FP32, EQFMM_FP32_BF16FAR               */
    double  origin[3];       /* lower corner of the box                                  */
    double  box;             /* side h > 0                                               */
    double  split_d;         /* split half-width d (Sec. 2.3); 0 selects leaf side/256;
                                must satisfy 0 < 2d < leaf side                          */
    double  node_shrink;     /* scale of the node lattice about the cell centre
                                (Sec. 4.1); 0 selects 1 (nodes on the faces)            */
    int64_t max_fragments;   /* capacity of the split charge set for the continuous
                                modes; 0 selects 2 * N + 4096                            */
} eqfmm_params;

typedef struct eqfmm_plan eqfmm_plan;

/* Build the host plan: node sets, shift matrices, the Coulomb matrices of
 * the bilinear form for every cell displacement, and (periodic modes) the
 * root operator, all in FP64 on the host.  *out receives the plan. */
int eqfmm_plan_create(const eqfmm_params *params, eqfmm_plan **out);

/* Bytes of device memory the plan needs (caller allocates, >= 256-aligned). */
int eqfmm_plan_device_bytes(const eqfmm_plan *plan, size_t *bytes);

/* Copy the plan's operators into the caller's device buffer (rounded to the
 * working precision).  Synchronises `stream`.  The buffer must outlive every
 * later call with this plan.  The first upload also creates, on the current
 * device, the plan's own non-blocking stream (default priority) and two
 * events: eqfmm_forward runs the near field there, concurrently with the far
 * field, and joins it back into the caller's stream before it returns. */
int eqfmm_plan_upload(eqfmm_plan *plan, void *dev_buf, size_t bytes, void *stream);

/* Bytes of workspace needed for n charges (an upper bound that includes the
 * fragment capacity of the continuous modes). */
int eqfmm_workspace_bytes(const eqfmm_plan *plan, int64_t n, size_t *bytes);

/* Forward evaluation (Sec. 2.2 steps 1-5 with Sec. 2.3 / Sec. 4.2).
 *   pos    [n][3] double, device; q [n] double, device.
 *   phi    [n] (float in FP32 modes, double in FP64 mode) or NULL.
 *   field  [n][3] (same type) or NULL: minus the exact gradient of the
 *          computed energy with respect to x_i, divided by q_i.
 *   energy device double scalar or NULL.
 *   ws     workspace of ws_bytes >= eqfmm_workspace_bytes(plan, n); it keeps
 *          the state that eqfmm_backward reads.
 * n = 0 is valid (energy 0). */
int eqfmm_forward(eqfmm_plan *plan, int64_t n, const double *pos, const double *q,
                  void *phi, void *field, double *energy,
                  void *ws, size_t ws_bytes, void *stream);

/* As eqfmm_forward, but never blocks: the data-dependent status (EQFMM_OK,
 * EQFMM_EBOX, EQFMM_ENEUTRAL, EQFMM_ENONFINITE or EQFMM_EWORKSPACE) is
 * written to *status, a device int32, when the enqueued work completes; the
 * return value covers only the errors found on the host (EINVAL, a
 * workspace smaller than eqfmm_workspace_bytes, EHIP).  eqfmm_backward may
 * follow on the same stream at once; its outputs are unspecified if *status
 * ends up non-zero.  For callers that enqueue many evaluations (serving
 * loops, graph capture) and check the status when they synchronise. */
int eqfmm_forward_async(eqfmm_plan *plan, int64_t n, const double *pos, const double *q,
                        void *phi, void *field, double *energy, int32_t *status,
                        void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the energy: given dL/dE (device double scalar), writes
 *   dEdx [n][3] = dL/dE * dE/dx_i  and  dEdq [n] = dL/dE * dE/dq_i
 * (float in FP32 modes, double in FP64), either may be NULL.  q must be the
 * charges of the preceding eqfmm_forward on the same workspace. */
int eqfmm_backward(eqfmm_plan *plan, int64_t n, const double *q, const double *grad_energy,
                   void *dEdx, void *dEdq, void *ws, size_t ws_bytes, void *stream);

/* Release the host plan (the device buffers stay the caller's). */
int eqfmm_plan_destroy(eqfmm_plan *plan);

const char *eqfmm_strerror(int code);

/* Stage timing with HIP events recorded on the stream each stage runs on.
 * `stages` is a bit mask (bit s times stage s, EQFMM_STAGES_ALL every stage,
 * 0 none); every launch of a timed stage is bracketed by two events, which
 * costs a few microseconds per pair, so a throughput measurement should time
 * only the stages it reports.  eqfmm_profile_read
 * synchronises and returns, for `stage` (EQFMM_STAGE_*), the summed kernel
 * time in ms, the number of launches, and the algorithmic flop and byte
 * counts of those launches (EQFMM_STAGE_M2L: one launch covers every
 * interaction level; two in the bf16 mode).  Enabling clears the totals. */
enum {
    EQFMM_STAGE_BIN = 0, EQFMM_STAGE_P2M = 1, EQFMM_STAGE_M2M = 2, EQFMM_STAGE_M2L = 3,
    EQFMM_STAGE_L2L = 4, EQFMM_STAGE_LEAF = 5, EQFMM_STAGE_GATHER = 6, EQFMM_STAGE_ADJOINT = 7,
    EQFMM_NUM_STAGES = 8, EQFMM_STAGES_ALL = (1 << 8) - 1
};
int eqfmm_profile_enable(eqfmm_plan *plan, int stages);
int eqfmm_profile_read(eqfmm_plan *plan, int stage, double *ms, int64_t *launches,
                       double *flops, double *bytes);

/* Library build information (architecture and version string). */
const char *eqfmm_version(void);

#ifdef __cplusplus
}
#endif
#endif
