// Internal declarations of the eqfmm library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "eqfmm.h"

namespace eqfmm {

constexpr int kMaxOrder = 7;
constexpr int kMaxPieces = kMaxOrder + 1;   // split pieces along one axis (odd n: n + 1)
constexpr int kNumOffsets = 343;            // 7^3 displacements between same-level cells
constexpr int kListLen = 192;               // interaction list (189) padded for the far-field kernels
constexpr int kHalo = 3;                    // halo cells around each level of the far-field input

// Geometry shared by every kernel (passed by value).
struct Geom {
    int n, n3, ns;        // order, n^3, stride of one cell's vector (n^3 rounded up to 16)
    int L, D;             // finest level, 2^L
    int boundary, periodic, continuous;
    double box, s_leaf, d;
    double origin[3];
};

// Device views of the uploaded plan.
struct DevOps {
    const void *t;          // working-precision unit nodes [n]
    const void *inv_den;    // working-precision Lagrange denominators [n]
    const double *t64;      // FP64 unit nodes [n]
    const double *seg64;    // FP64 split-segment nodes on [0,1] [n]
    const double *seg_den64;// FP64 split-segment Lagrange denominators [n]
    const void *G;          // child->parent shift matrices [2][n][n], G_b[j][i]
    const void *K;          // Coulomb matrices [343][n3][n3] at unit cell side
    const void *T;          // periodic root operator [n3][n3] at unit box side
    const void *Kmx;        // matrix-core operand layout of K (precision specific)
    const int *mxtab;       // interaction lists [level][parity][kListLen], packed
                            // (delta << 9) | oi: delta = source row - target row in
                            // the haloed layout of that level, oi = 0..342 the
                            // displacement's matrix
};

// Host plan (the public opaque type).
struct HostOps {
    std::vector<double> t, inv_den, seg, seg_den, G, K, T;
};

struct Profile {
    unsigned mask = 0;                // bit s: stage s is timed
    std::vector<hipEvent_t> pool;
    std::vector<int> stage_of;        // per event pair
    std::vector<double> flops_of, bytes_of;
    size_t used = 0;
    double ms[EQFMM_NUM_STAGES] = {};
    int64_t launches[EQFMM_NUM_STAGES] = {};
    double flops[EQFMM_NUM_STAGES] = {}, bytes[EQFMM_NUM_STAGES] = {};
};

// Workspace layout for a given N (byte offsets from the workspace base).
struct WsLayout {
    int64_t n = 0, fcap = 0, nleaf = 0;
    size_t hdr, cnt, fstart, smask, leafcnt, leafstart, cursor, scanblk;
    size_t su, sv, sw, sq, spar, sleaf;
    size_t gslot, gw, gdw;
    size_t phi, phipad, loc, loc2, sphi, snf, sfld, epart;
    size_t total;
    int64_t scan_blocks, e_blocks;
    std::vector<int64_t> lvl;     // first cell of each level in the Phi / L arrays
    std::vector<int64_t> plvl;    // first cell of each interaction level in the haloed Phi
};

struct WsHeader {
    int32_t flags;        // bit 0 out of box, bit 1 non-finite
    int32_t status;       // EQFMM_OK or the data-dependent error of the forward
    int64_t nfrag;        // total fragments (after the scan, before clamping to capacity)
    double qsum, qabs;    // neutrality check
    double energy;        // reduced energy (mirror of the output)
};

}  // namespace eqfmm

struct eqfmm_plan {
    eqfmm_params p;
    eqfmm::Geom g;
    eqfmm::HostOps h;
    std::vector<unsigned char> image;     // device image, built at create
    size_t off_t, off_den, off_t64, off_seg, off_segden, off_G, off_K, off_T, off_Kmx, off_mxtab;
    void *dev = nullptr;
    eqfmm::DevOps ops{};
    // forward state consumed by backward
    const void *last_ws = nullptr;
    int64_t last_n = -1, last_nfrag = 0;
    eqfmm::Profile prof;
    // the near field runs on a stream of its own, concurrent with the far
    // field; created with the plan's upload on the device in use then
    hipStream_t side = nullptr;
    hipEvent_t ev_bin = nullptr, ev_near = nullptr;
};

namespace eqfmm {

int build_host_ops(const eqfmm_params &p, const Geom &g, HostOps &h);
int build_image(eqfmm_plan *plan);
WsLayout ws_layout(const eqfmm_plan *plan, int64_t n);

// launchers (kernels.hip); all enqueue on `st`
// Enqueues the forward; its status code goes to the header and, if status
// is not NULL, to *status (device) when the work completes.
int run_forward(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi,
                void *field, double *energy, int *status, unsigned char *ws, const WsLayout &W, hipStream_t st);
int run_backward(eqfmm_plan *plan, int64_t n, const double *q, const double *gE, void *dEdx,
                 void *dEdq, unsigned char *ws, const WsLayout &W, hipStream_t st);

}  // namespace eqfmm
