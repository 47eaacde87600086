// Host side of the plan: FP64 operators of the method, the device image,
// the workspace layout, and the C ABI entry points.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "internal.h"

namespace eqfmm {

namespace {

constexpr double kPi = 3.14159265358979323846;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lagrange basis on the nodes x[0..n-1] evaluated at u (Sec. 2.1.1).
double lagrange(int n, const double *x, int i, double u)
{
    double num = 1.0, den = 1.0;
    for (int k = 0; k < n; ++k) {
        if (k == i) continue;
        num *= u - x[k];
        den *= x[i] - x[k];
    }
    return num / den;
}

// Interaction of a unit charge with the far periodic images (every image
// block outside the 3x3x3 block around the box) of a unit charge displaced
// by r, box side 1, tin-foil convention: the Ewald Green's function with the
// 27 nearest image terms removed.  Real-space part with alpha = 2.6 over
// images |m|_inf <= 4, reciprocal part over |k|_inf <= 9 (units of 2 pi).
double far_images(const double r[3])
{
    const double a = 2.6;
    const int R = 4, K = 9;
    double real = 0.0;
    for (int mx = -R; mx <= R; ++mx)
        for (int my = -R; my <= R; ++my)
            for (int mz = -R; mz <= R; ++mz) {
                const double dx = r[0] + mx, dy = r[1] + my, dz = r[2] + mz;
                const double rho = std::sqrt(dx * dx + dy * dy + dz * dz);
                const bool inner = std::abs(mx) <= 1 && std::abs(my) <= 1 && std::abs(mz) <= 1;
                if (!inner) real += std::erfc(a * rho) / rho;
                else real -= rho > 0.0 ? std::erf(a * rho) / rho : 2.0 * a / std::sqrt(kPi);
            }
    double recip = 0.0;
    for (int kx = -K; kx <= K; ++kx)
        for (int ky = -K; ky <= K; ++ky)
            for (int kz = -K; kz <= K; ++kz) {
                if (!kx && !ky && !kz) continue;
                const double k2 = 4.0 * kPi * kPi * (kx * kx + ky * ky + kz * kz);
                recip += std::exp(-k2 / (4.0 * a * a)) / k2 *
                         std::cos(2.0 * kPi * (kx * r[0] + ky * r[1] + kz * r[2]));
            }
    return real + 4.0 * kPi * recip - kPi / (a * a);
}

}  // namespace

int build_host_ops(const eqfmm_params &p, const Geom &g, HostOps &h)
{
    const int n = g.n, n3 = g.n3;
    const double sigma = p.node_shrink > 0.0 ? p.node_shrink : 1.0;
    h.t.resize(n);
    h.inv_den.resize(n);
    h.seg.resize(n);
    h.seg_den.resize(n);
    for (int a = 0; a < n; ++a) {
        h.seg[a] = double(a) / double(n - 1);
        h.t[a] = sigma * (h.seg[a] - 0.5) + 0.5;
    }
    for (int i = 0; i < n; ++i) {
        double d1 = 1.0, d2 = 1.0;
        for (int k = 0; k < n; ++k) {
            if (k == i) continue;
            d1 *= h.t[i] - h.t[k];
            d2 *= h.seg[i] - h.seg[k];
        }
        h.inv_den[i] = 1.0 / d1;
        h.seg_den[i] = 1.0 / d2;
    }
    // child -> parent shift (Sec. 2.1.6): G_b[j][i] = g_j((b + t_i) / 2)
    h.G.assign(2 * n * n, 0.0);
    for (int b = 0; b < 2; ++b)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                h.G[(b * n + j) * n + i] = lagrange(n, h.t.data(), j, 0.5 * (b + h.t[i]));
    // Coulomb matrices of the bilinear form, Eq. (14), per displacement o of
    // the source cell in cell units: K_o[a][b] = 1 / |t_a - t_b - o|.
    h.K.assign(size_t(kNumOffsets) * n3 * n3, 0.0);
    for (int oz = -3; oz <= 3; ++oz)
        for (int oy = -3; oy <= 3; ++oy)
            for (int ox = -3; ox <= 3; ++ox) {
                if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
                const int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
                double *Ko = &h.K[size_t(oi) * n3 * n3];
                for (int a = 0; a < n3; ++a)
                    for (int b = 0; b < n3; ++b) {
                        const double dx = h.t[a % n] - h.t[b % n] - ox;
                        const double dy = h.t[(a / n) % n] - h.t[(b / n) % n] - oy;
                        const double dz = h.t[a / (n * n)] - h.t[b / (n * n)] - oz;
                        Ko[size_t(a) * n3 + b] = 1.0 / std::sqrt(dx * dx + dy * dy + dz * dz);
                    }
            }
    // periodic root operator on the box's own lattice; node differences take
    // (2n-1)^3 distinct values, so evaluate the lattice sum once for each
    h.T.clear();
    if (g.periodic) {
        const int m = 2 * n - 1;
        std::vector<double> memo(size_t(m) * m * m);
        for (int e = 0; e < m * m * m; ++e) {
            const int ix = e % m - (n - 1), iy = (e / m) % m - (n - 1), iz = e / (m * m) - (n - 1);
            const double r[3] = {sigma * ix / double(n - 1), sigma * iy / double(n - 1),
                                 sigma * iz / double(n - 1)};
            memo[e] = far_images(r);
        }
        h.T.resize(size_t(n3) * n3);
        for (int a = 0; a < n3; ++a)
            for (int b = 0; b < n3; ++b) {
                const int ix = a % n - b % n + (n - 1);
                const int iy = (a / n) % n - (b / n) % n + (n - 1);
                const int iz = a / (n * n) - b / (n * n) + (n - 1);
                h.T[size_t(a) * n3 + b] = memo[ix + m * (iy + m * iz)];
            }
    }
    return EQFMM_OK;
}

namespace {

template <typename R>
void put(std::vector<unsigned char> &img, size_t off, const std::vector<double> &v)
{
    R *dst = reinterpret_cast<R *>(img.data() + off);
    for (size_t i = 0; i < v.size(); ++i) dst[i] = R(v[i]);
}

}  // namespace

// Matrix-core operand layout of the Coulomb matrices used by the far-field
// kernels; defined with those kernels.
size_t mx_layout_bytes(const Geom &g, int precision);
void mx_layout_fill(const Geom &g, int precision, const std::vector<double> &K, unsigned char *dst);

int build_image(eqfmm_plan *plan)
{
    const Geom &g = plan->g;
    const HostOps &h = plan->h;
    const int prec = plan->p.precision;
    const size_t rs = prec == EQFMM_FP64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    plan->off_t = take(rs * g.n);
    plan->off_den = take(rs * g.n);
    plan->off_t64 = take(sizeof(double) * g.n);
    plan->off_seg = take(sizeof(double) * g.n);
    plan->off_segden = take(sizeof(double) * g.n);
    plan->off_G = take(rs * h.G.size());
    plan->off_K = take(rs * h.K.size());
    plan->off_T = take(rs * std::max<size_t>(h.T.size(), 1));
    plan->off_Kmx = take(std::max<size_t>(mx_layout_bytes(g, prec), 1));
    plan->off_mxtab = take(sizeof(int32_t) * (g.L + 1) * 8 * kListLen);
    plan->image.assign(off, 0);
    // interaction list of a cell with parity p (cell index mod 2 per axis):
    // displacements in [-2-p, 3-p]^3 that are not adjacent.  The list is
    // ordered by the parity of the displacement: all targets of one parity
    // then read sources of a single parity class for ~24 consecutive
    // displacements, a set that stays in L2.  The 189 entries are padded to
    // kListLen with the displacement (0,0,0), whose matrix is zero.  Each
    // entry is stored per level as the row distance in that level's haloed
    // layout (side 2^l + 2 kHalo) and the matrix index.
    {
        int32_t *tab = reinterpret_cast<int32_t *>(plan->image.data() + plan->off_mxtab);
        for (int p = 0; p < 8; ++p) {
            const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
            int ox_[kListLen] = {}, oy_[kListLen] = {}, oz_[kListLen] = {};
            int m = 0;
            for (int q = 0; q < 8; ++q)
                for (int oz = -2 - pz; oz <= 3 - pz; ++oz)
                    for (int oy = -2 - py; oy <= 3 - py; ++oy)
                        for (int ox = -2 - px; ox <= 3 - px; ++ox) {
                            if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
                            if (((ox & 1) | ((oy & 1) << 1) | ((oz & 1) << 2)) != q) continue;
                            ox_[m] = ox;
                            oy_[m] = oy;
                            oz_[m] = oz;
                            ++m;
                        }
            for (int l = 0; l <= g.L; ++l) {
                const int64_t P = (int64_t(1) << l) + 2 * kHalo;
                for (int k = 0; k < kListLen; ++k) {
                    const int64_t delta = (oz_[k] * P + oy_[k]) * P + ox_[k];
                    const int oi = (ox_[k] + 3) + 7 * (oy_[k] + 3) + 49 * (oz_[k] + 3);
                    tab[(l * 8 + p) * kListLen + k] = int32_t(delta * 512 + oi);
                }
            }
        }
    }
    auto &img = plan->image;
    if (prec == EQFMM_FP64) {
        put<double>(img, plan->off_t, h.t);
        put<double>(img, plan->off_den, h.inv_den);
        put<double>(img, plan->off_G, h.G);
        put<double>(img, plan->off_K, h.K);
        put<double>(img, plan->off_T, h.T);
    } else {
        put<float>(img, plan->off_t, h.t);
        put<float>(img, plan->off_den, h.inv_den);
        put<float>(img, plan->off_G, h.G);
        put<float>(img, plan->off_K, h.K);
        put<float>(img, plan->off_T, h.T);
    }
    put<double>(img, plan->off_t64, h.t);
    put<double>(img, plan->off_seg, h.seg);
    put<double>(img, plan->off_segden, h.seg_den);
    mx_layout_fill(g, prec, h.K, img.data() + plan->off_Kmx);
    return EQFMM_OK;
}

WsLayout ws_layout(const eqfmm_plan *plan, int64_t n)
{
    const Geom &g = plan->g;
    const size_t rs = plan->p.precision == EQFMM_FP64 ? sizeof(double) : sizeof(float);
    WsLayout W;
    W.n = n;
    W.nleaf = int64_t(1) << (3 * g.L);
    if (g.continuous)
        W.fcap = plan->p.max_fragments > 0 ? plan->p.max_fragments : 2 * n + 4096;
    else
        W.fcap = n;
    // fragment indices are 32-bit
    W.fcap = std::min<int64_t>(std::max<int64_t>(W.fcap, 1), int64_t(INT32_MAX) - 1);
    W.lvl.resize(g.L + 2);
    W.lvl[0] = 0;
    for (int l = 0; l <= g.L; ++l) W.lvl[l + 1] = W.lvl[l] + (int64_t(1) << (3 * l));
    const int64_t ncells = W.lvl[g.L + 1];
    W.scan_blocks = (std::max<int64_t>(n, W.nleaf) + 1 + 1023) / 1024;
    W.e_blocks = std::max<int64_t>((n + 255) / 256, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    W.hdr = take(sizeof(WsHeader));
    W.cnt = take(4 * (n + 1));
    W.fstart = take(4 * (n + 1));
    W.smask = take(std::max<int64_t>(n, 1));
    W.leafcnt = take(4 * (W.nleaf + 1));
    W.leafstart = take(4 * (W.nleaf + 1));
    W.cursor = take(4 * W.nleaf);
    W.scanblk = take(4 * (W.scan_blocks + 1));
    // cell-local coordinates in double in every mode (close pairs)
    W.su = take(sizeof(double) * W.fcap);
    W.sv = take(sizeof(double) * W.fcap);
    W.sw = take(sizeof(double) * W.fcap);
    W.sq = take(rs * W.fcap);
    W.spar = take(4 * W.fcap);
    W.sleaf = take(4 * W.fcap);
    W.gslot = take(4 * W.fcap);
    // split weights and fragment potentials in double in every mode: along a
    // split axis the force is a short sum of large cancelling terms
    W.gw = take(sizeof(double) * W.fcap);
    W.gdw = take(sizeof(double) * 3 * W.fcap);
    W.phi = take(rs * ncells * g.ns);
    // the interaction levels again, each inside a halo of kHalo cells (zeros
    // in free space, periodic images otherwise): the far-field kernels read
    // every source of a displacement at one fixed row distance
    W.plvl.assign(g.L + 2, 0);
    int64_t pcells = 0;
    for (int l = g.periodic ? 1 : 2; l <= g.L; ++l) {
        const int64_t P = (int64_t(1) << l) + 2 * kHalo;
        W.plvl[l] = pcells;
        pcells += P * P * P;
    }
    W.plvl[g.L + 1] = pcells;
    W.phipad = take(rs * pcells * g.ns);
    W.loc = take(rs * ncells * g.ns);
    // second halves of the coarse levels' local vectors (levels below L)
    W.loc2 = take(rs * std::max<int64_t>(W.lvl[g.L], 1) * g.ns);
    W.sphi = take(sizeof(double) * W.fcap);
    W.snf = take(sizeof(double) * 3 * W.fcap);   // near-field sums before the far field is added
    W.sfld = take(rs * 3 * W.fcap);
    W.epart = take(sizeof(double) * W.e_blocks);
    W.total = off;
    return W;
}

}  // namespace eqfmm

using namespace eqfmm;

extern "C" {

const char *eqfmm_strerror(int code)
{
    switch (code) {
        case EQFMM_OK: return "ok";
        case EQFMM_EINVAL: return "invalid argument";
        case EQFMM_EBOX: return "position outside the box (free boundary)";
        case EQFMM_ENEUTRAL: return "periodic boundary needs a neutral charge set";
        case EQFMM_ENONFINITE: return "non-finite position or charge";
        case EQFMM_EWORKSPACE: return "workspace too small or fragment capacity exceeded";
        case EQFMM_EHIP: return "HIP runtime error";
        case EQFMM_ESTATE: return "backward without a matching forward";
        default: return "unknown error";
    }
}

const char *eqfmm_version(void) { return "eqfmm 0.1 gfx950"; }

int eqfmm_plan_create(const eqfmm_params *params, eqfmm_plan **out)
{
    if (!params || !out) return EQFMM_EINVAL;
    const eqfmm_params &p = *params;
    if (p.levels < 2 || p.levels > 8 || p.order < 2 || p.order > kMaxOrder) return EQFMM_EINVAL;
    if (p.boundary < 0 || p.boundary > 3 || p.precision < 0 || p.precision > 2) return EQFMM_EINVAL;
    if (!(p.box > 0.0) || !std::isfinite(p.box)) return EQFMM_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p.origin[a])) return EQFMM_EINVAL;
    if (p.node_shrink < 0.0 || p.node_shrink > 1.0 || p.max_fragments < 0) return EQFMM_EINVAL;
    eqfmm_plan *plan = new (std::nothrow) eqfmm_plan();
    if (!plan) return EQFMM_EINVAL;
    plan->p = p;
    Geom &g = plan->g;
    g.n = p.order;
    g.n3 = g.n * g.n * g.n;
    g.ns = (g.n3 + 15) & ~15;
    g.L = p.levels;
    g.D = 1 << g.L;
    g.boundary = p.boundary;
    g.periodic = p.boundary == EQFMM_PERIODIC || p.boundary == EQFMM_PERIODIC_CONTINUOUS;
    g.continuous = p.boundary == EQFMM_FREE_CONTINUOUS || p.boundary == EQFMM_PERIODIC_CONTINUOUS;
    g.box = p.box;
    g.s_leaf = p.box / double(g.D);
    g.d = p.split_d > 0.0 ? p.split_d : g.s_leaf / 256.0;
    for (int a = 0; a < 3; ++a) g.origin[a] = p.origin[a];
    if (!(2.0 * g.d < g.s_leaf)) { delete plan; return EQFMM_EINVAL; }
    int rc = build_host_ops(p, g, plan->h);
    if (rc == EQFMM_OK) rc = build_image(plan);
    if (rc != EQFMM_OK) { delete plan; return rc; }
    *out = plan;
    return EQFMM_OK;
}

int eqfmm_plan_device_bytes(const eqfmm_plan *plan, size_t *bytes)
{
    if (!plan || !bytes) return EQFMM_EINVAL;
    *bytes = plan->image.size();
    return EQFMM_OK;
}

int eqfmm_plan_upload(eqfmm_plan *plan, void *dev_buf, size_t bytes, void *stream)
{
    if (!plan || !dev_buf || bytes < plan->image.size()) return EQFMM_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return EQFMM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(dev_buf, plan->image.data(), plan->image.size(), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return EQFMM_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return EQFMM_EHIP;
    unsigned char *b = static_cast<unsigned char *>(dev_buf);
    plan->dev = dev_buf;
    plan->ops.t = b + plan->off_t;
    plan->ops.inv_den = b + plan->off_den;
    plan->ops.t64 = reinterpret_cast<const double *>(b + plan->off_t64);
    plan->ops.seg64 = reinterpret_cast<const double *>(b + plan->off_seg);
    plan->ops.seg_den64 = reinterpret_cast<const double *>(b + plan->off_segden);
    plan->ops.G = b + plan->off_G;
    plan->ops.K = b + plan->off_K;
    plan->ops.T = b + plan->off_T;
    plan->ops.Kmx = b + plan->off_Kmx;
    plan->ops.mxtab = reinterpret_cast<const int *>(b + plan->off_mxtab);
    if (!plan->side) {
        // default priority; non-blocking so that it never waits on the legacy stream by itself
        if (hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking) != hipSuccess) return EQFMM_EHIP;
        if (hipEventCreateWithFlags(&plan->ev_bin, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&plan->ev_near, hipEventDisableTiming) != hipSuccess)
            return EQFMM_EHIP;
    }
    return EQFMM_OK;
}

int eqfmm_workspace_bytes(const eqfmm_plan *plan, int64_t n, size_t *bytes)
{
    if (!plan || !bytes || n < 0 || n > (int64_t(1) << 30)) return EQFMM_EINVAL;
    *bytes = ws_layout(plan, n).total;
    return EQFMM_OK;
}

namespace {

int forward_common(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi, void *field,
                   double *energy, int32_t *status, void *ws, size_t ws_bytes, void *stream, bool wait)
{
    if (!plan || !plan->dev || n < 0 || n > (int64_t(1) << 30)) return EQFMM_EINVAL;
    if (n > 0 && (!pos || !q)) return EQFMM_EINVAL;
    if (!ws || (!wait && !status)) return EQFMM_EINVAL;
    WsLayout W = ws_layout(plan, n);
    if (ws_bytes < W.total) return EQFMM_EWORKSPACE;
    plan->last_ws = nullptr;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char *w = static_cast<unsigned char *>(ws);
    int rc = run_forward(plan, n, pos, q, phi, field, energy, status, w, W, st);
    if (rc == EQFMM_OK && wait) {
        int32_t code = 0;
        const WsHeader *hdr = reinterpret_cast<const WsHeader *>(w + W.hdr);
        if (hipMemcpyAsync(&code, &hdr->status, sizeof(code), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return EQFMM_EHIP;
        rc = code;
    }
    if (rc == EQFMM_OK) {
        plan->last_ws = ws;
        plan->last_n = n;
    }
    return rc;
}

}  // namespace

int eqfmm_forward(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi,
                  void *field, double *energy, void *ws, size_t ws_bytes, void *stream)
{
    return forward_common(plan, n, pos, q, phi, field, energy, nullptr, ws, ws_bytes, stream, true);
}

int eqfmm_forward_async(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi,
                        void *field, double *energy, int32_t *status, void *ws, size_t ws_bytes, void *stream)
{
    return forward_common(plan, n, pos, q, phi, field, energy, status, ws, ws_bytes, stream, false);
}

int eqfmm_backward(eqfmm_plan *plan, int64_t n, const double *q, const double *grad_energy,
                   void *dEdx, void *dEdq, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !plan->dev || !ws || !grad_energy || n < 0) return EQFMM_EINVAL;
    if (n > 0 && !q) return EQFMM_EINVAL;
    if (plan->last_ws != ws || plan->last_n != n) return EQFMM_ESTATE;
    WsLayout W = ws_layout(plan, n);
    if (ws_bytes < W.total) return EQFMM_EWORKSPACE;
    return run_backward(plan, n, q, grad_energy, dEdx, dEdq, static_cast<unsigned char *>(ws), W,
                        static_cast<hipStream_t>(stream));
}

int eqfmm_plan_destroy(eqfmm_plan *plan)
{
    if (!plan) return EQFMM_EINVAL;
    for (hipEvent_t e : plan->prof.pool) (void)hipEventDestroy(e);
    if (plan->ev_bin) (void)hipEventDestroy(plan->ev_bin);
    if (plan->ev_near) (void)hipEventDestroy(plan->ev_near);
    if (plan->side) (void)hipStreamDestroy(plan->side);
    delete plan;
    return EQFMM_OK;
}

int eqfmm_profile_enable(eqfmm_plan *plan, int stages)
{
    if (!plan) return EQFMM_EINVAL;
    Profile &P = plan->prof;
    P.mask = unsigned(stages) & ((1u << EQFMM_NUM_STAGES) - 1u);
    P.used = 0;
    P.stage_of.clear();
    P.flops_of.clear();
    P.bytes_of.clear();
    for (int s = 0; s < EQFMM_NUM_STAGES; ++s) {
        P.ms[s] = 0.0;
        P.launches[s] = 0;
        P.flops[s] = P.bytes[s] = 0.0;
    }
    return EQFMM_OK;
}

int eqfmm_profile_read(eqfmm_plan *plan, int stage, double *ms, int64_t *launches, double *flops,
                       double *bytes)
{
    if (!plan || stage < 0 || stage >= EQFMM_NUM_STAGES) return EQFMM_EINVAL;
    Profile &P = plan->prof;
    // fold the recorded event pairs into the totals
    for (size_t k = 0; k < P.stage_of.size(); ++k) {
        hipEvent_t a = P.pool[2 * k], b = P.pool[2 * k + 1];
        if (hipEventSynchronize(b) != hipSuccess) return EQFMM_EHIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, a, b) != hipSuccess) return EQFMM_EHIP;
        const int s = P.stage_of[k];
        P.ms[s] += t;
        P.launches[s] += 1;
        P.flops[s] += P.flops_of[k];
        P.bytes[s] += P.bytes_of[k];
    }
    P.stage_of.clear();
    P.flops_of.clear();
    P.bytes_of.clear();
    P.used = 0;
    if (ms) *ms = P.ms[stage];
    if (launches) *launches = P.launches[stage];
    if (flops) *flops = P.flops[stage];
    if (bytes) *bytes = P.bytes[stage];
    return EQFMM_OK;
}

}  // extern "C"
