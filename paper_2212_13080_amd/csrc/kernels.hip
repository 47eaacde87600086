// gfx950 kernels of the replacement FMM and the forward / adjoint drivers.
//
// Data layout in HBM (one workspace, see ws_layout):
//   - charges are split (continuous modes) into "fragments"; fragments are
//     counting-sorted by finest cell (row-major cell index, x fastest), and
//     the sorted arrays hold cell-local coordinates u in [0,1]^3, q * w, the
//     owning charge and the cell;
//   - Phi and the local vectors L of every level are [cell][ns] rows
//     (ns = n^3 rounded up to 16, zero padded), level 0 first;
//   - per-fragment potential / field are written in sorted order and
//     gathered back to the charges through the fragment -> slot map.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace eqfmm {

#define EQ_CHECK(x)                                  \
    do {                                             \
        if ((x) != hipSuccess) return EQFMM_EHIP;    \
    } while (0)

// ------------------------------------------------------------------ timing

namespace {

int prof_begin(eqfmm_plan *plan, hipStream_t st, int stage)
{
    Profile &P = plan->prof;
    if (!((P.mask >> stage) & 1u)) return -1;
    const size_t k = P.stage_of.size();
    while (P.pool.size() < 2 * (k + 1)) {
        hipEvent_t e;
        // timing only: no system-scope fence, which would write back and
        // invalidate the caches under the kernels that follow
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        P.pool.push_back(e);
    }
    if (hipEventRecord(P.pool[2 * k], st) != hipSuccess) return -1;
    P.stage_of.push_back(-1);
    P.flops_of.push_back(0.0);
    P.bytes_of.push_back(0.0);
    return int(k);
}

void prof_end(eqfmm_plan *plan, hipStream_t st, int k, int stage, double flops, double bytes)
{
    if (k < 0) return;
    Profile &P = plan->prof;
    (void)hipEventRecord(P.pool[2 * k + 1], st);
    P.stage_of[k] = stage;
    P.flops_of[k] = flops;
    P.bytes_of[k] = bytes;
}

}  // namespace

// ------------------------------------------------------------- device math

template <int N> struct Ord {
    static constexpr int N3 = N * N * N;
    static constexpr int NS = (N3 + 15) & ~15;
    static constexpr int TPC = ((NS + 63) / 64) * 64;   // threads per cell vector
};

// Lagrange basis of the unit nodes t at u (Sec. 2.1.1), values only.
template <int N, typename R>
__device__ __forceinline__ void lag_vals(const R *t, const R *den, R u, R *g)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R p = den[i];
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k != i) p *= (u - t[k]);
        g[i] = p;
    }
}

// values and derivatives (product rule accumulated alongside)
template <int N, typename R>
__device__ __forceinline__ void lag_vals_der(const R *t, const R *den, R u, R *g, R *dg)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R p = R(1), dp = R(0);
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k != i) {
                dp = dp * (u - t[k]) + p;
                p = p * (u - t[k]);
            }
        g[i] = den[i] * p;
        dg[i] = den[i] * dp;
    }
}

// Position relative to the origin: periodic wrap, or box check (free).
// Returns error bits (1 outside, 2 non-finite) and a safe in-range value.
__device__ __forceinline__ int box_coord(const Geom &g, double x, int a, double &v)
{
    v = x - g.origin[a];
    if (!isfinite(v)) {
        v = 0.0;
        return 2;
    }
    if (g.periodic) {
        v -= g.box * floor(v / g.box);
        if (v >= g.box) v -= g.box;
        if (v < 0.0) v = 0.0;
        return 0;
    }
    if (v < 0.0 || v > g.box) {
        v = fmin(fmax(v, 0.0), g.box);
        return 1;
    }
    return 0;
}

// Pieces of one axis (Sec. 2.3, Sec. 4.2): the charge itself, or the n
// equally spaced points of the segment of length 2d centred on the nearby
// face, weighted by the segment's Lagrange basis; the point on the face
// (odd n) is halved into the two cells; cells wrap in periodic modes.
template <int N>
struct Pieces {
    int cnt;
    int cell[N + 1];
    double u[N + 1], om[N + 1], dom[N + 1];
};

template <int N, bool WEIGHTS>
__device__ __forceinline__ void axis_pieces(const Geom &g, const double *seg, const double *segden,
                                            double v, Pieces<N> &P)
{
    const double s = g.s_leaf, d = g.d;
    int c = int(floor(v / s));
    c = c < 0 ? 0 : (c >= g.D ? g.D - 1 : c);
    const double dlo = v - c * s, dhi = (c + 1) * s - v;
    int fb = -1;
    if (g.continuous) {
        if (dlo < d && (g.periodic || c > 0)) fb = c;
        else if (dhi < d && (g.periodic || c < g.D - 1)) fb = c + 1;
    }
    if (fb < 0) {
        P.cnt = 1;
        P.cell[0] = c;
        if (WEIGHTS) {
            P.u[0] = v / s - c;
            P.om[0] = 1.0;
            P.dom[0] = 0.0;
        }
        return;
    }
    const double b = fb * s;
    const double tau = (v - (b - d)) / (2.0 * d);
    int m = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double w = 0.0, dw = 0.0;
        if (WEIGHTS) {
            double p = 1.0, dp = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j)
                if (j != k) {
                    dp = dp * (tau - seg[j]) + p;
                    p = p * (tau - seg[j]);
                }
            w = segden[k] * p;
            dw = segden[k] * dp / (2.0 * d);
        }
        const double off = d * (2.0 * k / double(N - 1) - 1.0);   // piece - face
        const int side = 2 * k < N - 1 ? 0 : (2 * k > N - 1 ? 1 : 2);
        for (int e = 0; e < (side == 2 ? 2 : 1); ++e) {
            const int up = side == 2 ? e : side;
            int cell = up ? fb : fb - 1;
            if (cell < 0) cell += g.D;
            if (cell >= g.D) cell -= g.D;
            P.cell[m] = cell;
            if (WEIGHTS) {
                const double fr = side == 2 ? 0.5 : 1.0;
                P.u[m] = side == 2 ? double(1 - up) : (up ? off / s : 1.0 + off / s);
                P.om[m] = fr * w;
                P.dom[m] = fr * dw;
            }
            ++m;
        }
    }
    P.cnt = m;
}

// Finest cell along one axis and whether the charge is split there (the
// same test as axis_pieces, without the pieces).
__device__ __forceinline__ bool axis_split(const Geom &g, double v, int &c)
{
    const double s = g.s_leaf, d = g.d;
    c = int(floor(v / s));
    c = c < 0 ? 0 : (c >= g.D ? g.D - 1 : c);
    if (!g.continuous) return false;
    const double dlo = v - c * s, dhi = (c + 1) * s - v;
    return (dlo < d && (g.periodic || c > 0)) || (dhi < d && (g.periodic || c < g.D - 1));
}

// ------------------------------------------------------------ a1/a2: bin

// Clears the header, the per-cell counts and the cursors of one forward.
__global__ void __launch_bounds__(256) k_clear(WsHeader *hdr, int *leafcnt, int *cursor, int64_t nleaf)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i <= nleaf) leafcnt[i] = 0;
    if (i < nleaf) cursor[i] = 0;
    if (i == 0) *hdr = WsHeader{};
}

template <int N>
__global__ void __launch_bounds__(256) k_count(Geom g, const double *seg, int64_t n,
                                               const double *pos, const double *q, int *cnt, int *fstart,
                                               unsigned char *smask, int *leafcnt, WsHeader *hdr)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double qs = 0.0, qa = 0.0;
    if (i < n) {
        int flags = 0;
        double v[3];
        int c[3];
        bool split = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            flags |= box_coord(g, pos[3 * i + a], a, v[a]);
            split |= axis_split(g, v[a], c[a]);
        }
        const double qi = q[i];
        if (!isfinite(qi)) flags |= 2;
        if (!split) {   // one piece, in cell c (every charge of the unsplit modes)
            if (g.continuous) cnt[i] = 1;
            else {
                fstart[i] = int(i);   // one fragment per charge: the prefix sums are the identity
                if (i == n - 1) fstart[n] = int(n);
            }
            smask[i] = 0;
            atomicAdd(&leafcnt[c[0] + int64_t(g.D) * (c[1] + int64_t(g.D) * c[2])], 1);
        } else {
            Pieces<N> P[3];
            for (int a = 0; a < 3; ++a) axis_pieces<N, false>(g, seg, nullptr, v[a], P[a]);
            cnt[i] = P[0].cnt * P[1].cnt * P[2].cnt;
            smask[i] = (P[0].cnt > 1) | ((P[1].cnt > 1) << 1) | ((P[2].cnt > 1) << 2);
            for (int kz = 0; kz < P[2].cnt; ++kz)
                for (int ky = 0; ky < P[1].cnt; ++ky)
                    for (int kx = 0; kx < P[0].cnt; ++kx) {
                        const int64_t leaf =
                            P[0].cell[kx] + int64_t(g.D) * (P[1].cell[ky] + int64_t(g.D) * P[2].cell[kz]);
                        atomicAdd(&leafcnt[leaf], 1);
                    }
        }
        if (flags) atomicOr(&hdr->flags, flags);
        if (isfinite(qi)) {
            qs = qi;
            qa = fabs(qi);
        }
    }
    if (g.periodic) {
        __shared__ double rs[256], ra[256];
        rs[threadIdx.x] = qs;
        ra[threadIdx.x] = qa;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                rs[threadIdx.x] += rs[threadIdx.x + w];
                ra[threadIdx.x] += ra[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            atomicAdd(&hdr->qsum, rs[0]);
            atomicAdd(&hdr->qabs, ra[0]);
        }
    }
}

template <int N, typename R>
__global__ void __launch_bounds__(256) k_emit(Geom g, const double *seg, const double *segden,
                                              int64_t n, const double *pos, const double *q,
                                              const int *fstart, const int *leafstart, int *cursor,
                                              double *su, double *sv, double *sw, R *sq, int *spar,
                                              int *sleaf, int *gslot, double *gw, double *gdw, int64_t fcap)
{
    // Fragments past the capacity fcap are dropped (the forward then reports
    // EQFMM_EWORKSPACE); the prefix sums are clamped to fcap, so every index
    // read later stays in range.
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[3];
    int c[3];
    bool split = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        box_coord(g, pos[3 * i + a], a, v[a]);
        split |= axis_split(g, v[a], c[a]);
    }
    const double qi = q[i];
    int f = fstart[i];
    if (!split) {   // one piece of weight 1 in cell c (as axis_pieces gives it)
        // only the owner goes to the sorted slot here; k_fill writes the
        // rest of the slot in slot order (coalesced stores)
        const int leaf = c[0] + g.D * (c[1] + g.D * c[2]);
        const int slot = leafstart[leaf] + atomicAdd(&cursor[leaf], 1);
        if (slot < fcap) spar[slot] = int(i);
        // an unsplit charge's weight is 1 and its weight gradient 0: the
        // gather and the adjoint take them from its empty split mask
        if (f < fcap) gslot[f] = slot < fcap ? slot : 0;
        return;
    }
    Pieces<N> P[3];
    for (int a = 0; a < 3; ++a) axis_pieces<N, true>(g, seg, segden, v[a], P[a]);
    for (int kz = 0; kz < P[2].cnt; ++kz)
        for (int ky = 0; ky < P[1].cnt; ++ky)
            for (int kx = 0; kx < P[0].cnt; ++kx, ++f) {
                const int leaf = P[0].cell[kx] + g.D * (P[1].cell[ky] + g.D * P[2].cell[kz]);
                const int slot = leafstart[leaf] + atomicAdd(&cursor[leaf], 1);
                const double ox = P[0].om[kx], oy = P[1].om[ky], oz = P[2].om[kz];
                const double w = ox * oy * oz;
                if (slot < fcap) {
                    su[slot] = P[0].u[kx];
                    sv[slot] = P[1].u[ky];
                    sw[slot] = P[2].u[kz];
                    sq[slot] = R(qi * w);
                    spar[slot] = int(i);
                    sleaf[slot] = leaf;
                }
                if (f < fcap) {
                    gslot[f] = slot < fcap ? slot : 0;
                    gw[f] = w;
                    gdw[3 * int64_t(f) + 0] = P[0].dom[kx] * oy * oz;
                    gdw[3 * int64_t(f) + 1] = ox * P[1].dom[ky] * oz;
                    gdw[3 * int64_t(f) + 2] = ox * oy * P[2].dom[kz];
                }
            }
}

// The sorted slots of unsplit charges, in slot order: the owner written by
// k_emit gives the charge, whose cell-local coordinates, charge and cell are
// computed again exactly as k_emit computes them.  Split charges' slots were
// written whole by k_emit.  nfrag: the (clamped) slot count on the device.
template <typename R>
__global__ void __launch_bounds__(256) k_fill(Geom g, const int *nfrag, const double *pos, const double *q,
                                              const unsigned char *smask, const int *spar, double *su, double *sv,
                                              double *sw, R *sq, int *sleaf)
{
    const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (slot >= *nfrag) return;
    const int i = spar[slot];
    if (smask[i]) return;
    double v[3];
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        box_coord(g, pos[3 * int64_t(i) + a], a, v[a]);
        axis_split(g, v[a], c[a]);
    }
    const double s = g.s_leaf;
    su[slot] = v[0] / s - c[0];
    sv[slot] = v[1] / s - c[1];
    sw[slot] = v[2] / s - c[2];
    sq[slot] = R(q[i]);
    sleaf[slot] = c[0] + g.D * (c[1] + g.D * c[2]);
}

// ------------------------------------------------------------- prefix sums

// exclusive scan of in[0..len) into out[0..len], out[len] = total
__global__ void __launch_bounds__(256) k_scan_local(const int *in, int *out, int64_t len, int *blk)
{
    __shared__ int sh[256];
    const int64_t base = int64_t(blockIdx.x) * 1024 + threadIdx.x * 4;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < len ? in[base + k] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const int add = threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - s;
    for (int k = 0; k < 4; ++k) {
        if (base + k < len) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) blk[blockIdx.x] = sh[255];
}

__global__ void __launch_bounds__(1024) k_scan_blocks(int *blk, int64_t nb)
{
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const int v = i < nb ? blk[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int w = 1; w < 1024; w <<= 1) {
            const int add = threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) blk[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[nb] = carry;
}

// Adds the block offsets; every prefix (and the total in out[len]) is
// clamped to clampv, and the unclamped total goes to *total.
__global__ void __launch_bounds__(256) k_scan_add(int *out, int64_t len, const int *blk, int64_t nb, int clampv,
                                                  int64_t *total)
{
    const int64_t base = int64_t(blockIdx.x) * 1024 + threadIdx.x * 4;
    const int add = blk[blockIdx.x];
    for (int k = 0; k < 4; ++k)
        if (base + k < len) {
            const int v = out[base + k] + add;
            out[base + k] = v < clampv ? v : clampv;
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int tot = blk[nb];
        out[len] = tot < clampv ? tot : clampv;
        if (total) *total = tot;
    }
}

// exclusive prefix sums of in[0, len) into out[0, len], clamped to clampv
int scan(const int *in, int *out, int64_t len, int *blk, int clampv, int64_t *total, hipStream_t st)
{
    const int64_t nb = (len + 1023) / 1024;
    if (nb == 0) return EQFMM_EINVAL;
    k_scan_local<<<dim3(unsigned(nb)), 256, 0, st>>>(in, out, len, blk);
    k_scan_blocks<<<1, 1024, 0, st>>>(blk, nb);
    k_scan_add<<<dim3(unsigned(nb)), 256, 0, st>>>(out, len, blk, nb, clampv, total);
    EQ_CHECK(hipGetLastError());
    return EQFMM_OK;
}

// --------------------------------------------------------- a3: replacement

// A workgroup owns CPB consecutive cells, whose charges are one contiguous
// range.  The charges are taken a chunk of blockDim.x at a time: each thread
// evaluates the Lagrange basis of one charge along the three axes into LDS,
// then the thread of coefficient a = i + n j + n^2 k of a cell adds
// q g_i(u) g_j(v) g_k(w) over the charges of its cell in the chunk.
template <int N, typename R>
__global__ void __launch_bounds__(512) k_p2m(const R *t_, const R *den_, int64_t nleaf,
                                             const int *leafstart, const double *su, const double *sv,
                                             const double *sw, const R *sq, R *phiL)
{
    using O = Ord<N>;
    constexpr int CPB = O::TPC >= 256 ? 1 : 256 / O::TPC;
    constexpr int CHK = CPB * O::TPC;   // threads per workgroup = charges per chunk
    __shared__ R gb[3][N][CHK];
    __shared__ R qs[CHK];
    const int cl = threadIdx.x / O::TPC, a = threadIdx.x % O::TPC;
    const int64_t cb = int64_t(blockIdx.x) * CPB;
    const int64_t ce = cb + CPB < nleaf ? cb + CPB : nleaf;
    const int64_t c = cb + cl;
    const int P0 = leafstart[cb], P1 = leafstart[ce];
    const bool mine = c < nleaf && a < O::N3;
    const int p0 = mine ? leafstart[c] : 0, p1 = mine ? leafstart[c + 1] : 0;
    R t[N], den[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        t[k] = t_[k];
        den[k] = den_[k];
    }
    const int i = a % N, j = (a / N) % N, k = a / (N * N);
    R acc = R(0);
    for (int q0 = P0; q0 < P1; q0 += CHK) {
        const int p = q0 + int(threadIdx.x);
        if (p < P1) {
            const R uvw[3] = {R(su[p]), R(sv[p]), R(sw[p])};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    R g = den[b];
#pragma unroll
                    for (int m = 0; m < N; ++m)
                        if (m != b) g *= uvw[ax] - t[m];
                    gb[ax][b][threadIdx.x] = g;
                }
            qs[threadIdx.x] = sq[p];
        }
        __syncthreads();
        if (mine) {
            const int lo = (p0 > q0 ? p0 : q0) - q0, hi = (p1 < q0 + CHK ? p1 : q0 + CHK) - q0;
            for (int e = lo; e < hi; ++e) acc += qs[e] * gb[0][i][e] * gb[1][j][e] * gb[2][k][e];
        }
        __syncthreads();
    }
    if (c < nleaf && a < O::NS) phiL[c * O::NS + a] = mine ? acc : R(0);
}

// -------------------------------------------------------- a4: shift upward

template <int N, typename R>
__global__ void __launch_bounds__(Ord<N>::TPC) k_m2m(const R *G, int Dl, const R *phic, R *phip)
{
    using O = Ord<N>;
    constexpr int N3 = O::N3;
    __shared__ R ch[8 * N3], tz[4 * N3], ty[2 * N3], Gs[2 * N * N];
    const int Dp = Dl >> 1;
    const int64_t P = blockIdx.x;
    const int X = int(P % Dp), Y = int((P / Dp) % Dp), Z = int(P / (int64_t(Dp) * Dp));
    for (int e = threadIdx.x; e < 8 * N3; e += blockDim.x) {
        const int b = e / N3, a = e % N3;
        const int64_t c = (2 * X + (b & 1)) + int64_t(Dl) * ((2 * Y + ((b >> 1) & 1)) +
                                                          int64_t(Dl) * (2 * Z + (b >> 2)));
        ch[e] = phic[c * O::NS + a];
    }
    for (int e = threadIdx.x; e < 2 * N * N; e += blockDim.x) Gs[e] = G[e];
    __syncthreads();
    // z: for each (bx,by), sum the two bz children shifted along z
    for (int o = threadIdx.x; o < 4 * N3; o += blockDim.x) {
        const int pr = o / N3, e = o % N3;
        const int i1 = e % N, i2 = (e / N) % N, j3 = e / (N * N);
        R acc = R(0);
        for (int bz = 0; bz < 2; ++bz)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3)
                acc += Gs[(bz * N + j3) * N + i3] * ch[(pr + 4 * bz) * N3 + i1 + N * i2 + N * N * i3];
        tz[o] = acc;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 2 * N3; o += blockDim.x) {
        const int bx = o / N3, e = o % N3;
        const int i1 = e % N, j2 = (e / N) % N, j3 = e / (N * N);
        R acc = R(0);
        for (int by = 0; by < 2; ++by)
#pragma unroll
            for (int i2 = 0; i2 < N; ++i2)
                acc += Gs[(by * N + j2) * N + i2] * tz[(bx + 2 * by) * N3 + i1 + N * i2 + N * N * j3];
        ty[o] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < O::NS; e += blockDim.x) {
        R acc = R(0);
        if (e < N3) {
            const int j1 = e % N, j2 = (e / N) % N, j3 = e / (N * N);
            for (int bx = 0; bx < 2; ++bx)
#pragma unroll
                for (int i1 = 0; i1 < N; ++i1)
                    acc += Gs[(bx * N + j1) * N + i1] * ty[bx * N3 + i1 + N * j2 + N * N * j3];
        }
        phip[P * O::NS + e] = acc;
    }
}

// ------------------------------------------------------ a6: shift downward

template <int N, typename R>
__global__ void __launch_bounds__(Ord<N>::TPC) k_l2l(const R *G, int Dl, const R *locp, const R *locp2, R *locc,
                                                     const R *locc2)
{
    using O = Ord<N>;
    constexpr int N3 = O::N3;
    __shared__ R lp[N3], ux[2 * N3], uy[4 * N3], Gs[2 * N * N];
    const int Dp = Dl >> 1;
    const int64_t P = blockIdx.x;
    const int X = int(P % Dp), Y = int((P / Dp) % Dp), Z = int(P / (int64_t(Dp) * Dp));
    // locp2 / locc2 (may be null): second halves of the far field
    for (int e = threadIdx.x; e < N3; e += blockDim.x)
        lp[e] = locp2 ? locp[P * O::NS + e] + locp2[P * O::NS + e] : locp[P * O::NS + e];
    for (int e = threadIdx.x; e < 2 * N * N; e += blockDim.x) Gs[e] = G[e];
    __syncthreads();
    // Psi_child(v) = Psi_parent(shift(v)): L_child = (G_bx x G_by x G_bz)^T L_parent
    for (int o = threadIdx.x; o < 2 * N3; o += blockDim.x) {
        const int bx = o / N3, e = o % N3;
        const int i1 = e % N, j2 = (e / N) % N, j3 = e / (N * N);
        R acc = R(0);
#pragma unroll
        for (int j1 = 0; j1 < N; ++j1) acc += Gs[(bx * N + j1) * N + i1] * lp[j1 + N * j2 + N * N * j3];
        ux[o] = acc;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 4 * N3; o += blockDim.x) {
        const int pr = o / N3, e = o % N3, bx = pr & 1, by = pr >> 1;
        const int i1 = e % N, i2 = (e / N) % N, j3 = e / (N * N);
        R acc = R(0);
#pragma unroll
        for (int j2 = 0; j2 < N; ++j2) acc += Gs[(by * N + j2) * N + i2] * ux[bx * N3 + i1 + N * j2 + N * N * j3];
        uy[o] = acc;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 8 * O::NS; o += blockDim.x) {
        const int b = o / O::NS, e = o % O::NS;
        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
        if (e >= N3) continue;
        const int i1 = e % N, i2 = (e / N) % N, i3 = e / (N * N);
        R acc = R(0);
#pragma unroll
        for (int j3 = 0; j3 < N; ++j3)
            acc += Gs[(bz * N + j3) * N + i3] * uy[(bx + 2 * by) * N3 + i1 + N * i2 + N * N * j3];
        const int64_t c = (2 * X + bx) + int64_t(Dl) * ((2 * Y + by) + int64_t(Dl) * (2 * Z + bz));
        const R own = locc2 ? locc[c * O::NS + e] + locc2[c * O::NS + e] : locc[c * O::NS + e];
        locc[c * O::NS + e] = own + acc;
    }
}

// periodic root: far images of the whole box acting on its own lattice (stores L_0)
template <typename R>
__global__ void __launch_bounds__(256) k_root(const R *T, int n3, R inv_box, const R *phi0, R *loc0)
{
    for (int a = threadIdx.x; a < n3; a += blockDim.x) {
        R acc = R(0);
        for (int b = 0; b < n3; ++b) acc += T[a * n3 + b] * phi0[b];
        loc0[a] = inv_box * acc;
    }
}

// -------------------------------------------------- a9 + a10: gather, energy

template <typename R>
__global__ void __launch_bounds__(256) k_gather(int64_t n, const double *q, const int *fstart,
                                                const unsigned char *smask, const int *gslot,
                                                const double *gw, const double *gdw, const double *sphi,
                                                const R *sfld, R *phi_out, R *fld_out, double *epart)
{
    __shared__ double red[256];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        const int f0 = fstart[i], f1 = fstart[i + 1];
        const int mask = smask[i];
        // accumulated in double: along split axes the terms cancel heavily
        double ph = 0.0, fe[3] = {0.0, 0.0, 0.0};
        for (int f = f0; f < f1; ++f) {
            const int sl = gslot[f];
            const double w = mask ? gw[f] : 1.0, pv = sphi[sl];
            ph += w * pv;
            for (int a = 0; a < 3; ++a) {
                if (mask & (1 << a)) fe[a] -= gdw[3 * int64_t(f) + a] * pv;
                else fe[a] += w * double(sfld[3 * int64_t(sl) + a]);
            }
        }
        if (phi_out) phi_out[i] = R(ph);
        if (fld_out)
            for (int a = 0; a < 3; ++a) fld_out[3 * i + a] = R(fe[a]);
        e = q[i] * ph;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

// Total energy, and the forward's status from the header: non-finite input,
// a position outside the box, a non-neutral periodic set, or more fragments
// than the capacity (in that order).
__global__ void __launch_bounds__(256) k_energy(const double *epart, int64_t nb, double *energy,
                                                WsHeader *hdr, int periodic, int64_t fcap, int *status)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) s += epart[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hdr->energy = 0.5 * red[0];
        if (energy) *energy = 0.5 * red[0];
        const int f = hdr->flags;
        int code = EQFMM_OK;
        if (f & 2) code = EQFMM_ENONFINITE;
        else if (f & 1) code = EQFMM_EBOX;
        else if (periodic && !(fabs(hdr->qsum) <= 1e-10 * hdr->qabs)) code = EQFMM_ENEUTRAL;
        else if (hdr->nfrag > fcap) code = EQFMM_EWORKSPACE;
        hdr->status = code;
        if (status) *status = code;
    }
}

// Adjoint of the energy with respect to positions and charges: the fragments
// of a charge sit at fixed points along its split axes while their weights
// follow the charge, and move with it along the other axes.
template <typename R>
__global__ void __launch_bounds__(256) k_adjoint(int64_t n, const double *q, const double *gE,
                                                 const int *fstart, const unsigned char *smask,
                                                 const int *gslot, const double *gw, const double *gdw,
                                                 const double *sphi, const R *sfld, R *dEdx, R *dEdq)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ge = *gE;
    const int f0 = fstart[i], f1 = fstart[i + 1];
    const int mask = smask[i];
    double ph = 0.0, gx[3] = {0.0, 0.0, 0.0};
    for (int f = f0; f < f1; ++f) {
        const int sl = gslot[f];
        const double w = mask ? gw[f] : 1.0, pv = sphi[sl];
        ph += w * pv;
        for (int a = 0; a < 3; ++a) {
            if (mask & (1 << a)) gx[a] += gdw[3 * int64_t(f) + a] * pv;
            else gx[a] -= w * double(sfld[3 * int64_t(sl) + a]);
        }
    }
    if (dEdq) dEdq[i] = R(ge * ph);
    if (dEdx)
        for (int a = 0; a < 3; ++a) dEdx[3 * i + a] = R(ge * q[i] * gx[a]);
}

// ------------------------------------------------------------------ drivers

namespace {

template <typename R> struct Ws {
    WsHeader *hdr;
    int *cnt, *fstart, *leafcnt, *leafstart, *cursor, *scanblk, *spar, *sleaf, *gslot;
    unsigned char *smask;
    R *sq, *phi, *phipad, *loc, *loc2, *sfld;
    double *su, *sv, *sw, *gw, *gdw, *sphi, *snf, *epart;
};

template <typename R> Ws<R> views(unsigned char *b, const WsLayout &W)
{
    Ws<R> v;
    v.hdr = reinterpret_cast<WsHeader *>(b + W.hdr);
    v.cnt = reinterpret_cast<int *>(b + W.cnt);
    v.fstart = reinterpret_cast<int *>(b + W.fstart);
    v.smask = b + W.smask;
    v.leafcnt = reinterpret_cast<int *>(b + W.leafcnt);
    v.leafstart = reinterpret_cast<int *>(b + W.leafstart);
    v.cursor = reinterpret_cast<int *>(b + W.cursor);
    v.scanblk = reinterpret_cast<int *>(b + W.scanblk);
    v.su = reinterpret_cast<double *>(b + W.su);
    v.sv = reinterpret_cast<double *>(b + W.sv);
    v.sw = reinterpret_cast<double *>(b + W.sw);
    v.sq = reinterpret_cast<R *>(b + W.sq);
    v.spar = reinterpret_cast<int *>(b + W.spar);
    v.sleaf = reinterpret_cast<int *>(b + W.sleaf);
    v.gslot = reinterpret_cast<int *>(b + W.gslot);
    v.gw = reinterpret_cast<double *>(b + W.gw);
    v.gdw = reinterpret_cast<double *>(b + W.gdw);
    v.phi = reinterpret_cast<R *>(b + W.phi);
    v.phipad = reinterpret_cast<R *>(b + W.phipad);
    v.loc = reinterpret_cast<R *>(b + W.loc);
    v.loc2 = reinterpret_cast<R *>(b + W.loc2);
    v.sphi = reinterpret_cast<double *>(b + W.sphi);
    v.snf = reinterpret_cast<double *>(b + W.snf);
    v.sfld = reinterpret_cast<R *>(b + W.sfld);
    v.epart = reinterpret_cast<double *>(b + W.epart);
    return v;
}

unsigned blocks(int64_t work, int per) { return unsigned((work + per - 1) / per); }

}  // namespace

// near field, and far field at the charges (near.hip)
template <typename R>
int launch_p2p(const eqfmm_plan *plan, int64_t n, int64_t fcap, const int *leafstart, const double *su,
               const double *sv, const double *sw, const R *sq, const int *spar, const int *sleaf,
               const unsigned char *smask, double *sphi, double *snf, hipStream_t st);
template <int N, typename R>
int launch_l2p(const eqfmm_plan *plan, int64_t fcap, const int *leafstart, const R *t, const R *den,
               const double *su, const double *sv, const double *sw, const int *spar, const int *sleaf,
               const unsigned char *smask, const R *locL, double *sphi, const double *snf, R *sfld, hipStream_t st);

// far field (declared here, defined with the matrix-core kernels in m2l.hip):
// the haloed copy of Phi at levels lmin..lmax, then the products of every
// interaction level
template <typename R>
int launch_m2l_pad(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const R *phi,
                   R *phipad, hipStream_t st);
template <typename R>
int launch_m2l(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const R *phipad,
               R *loc, R *loc2, hipStream_t st);
// levels (bit l) whose local vectors the far field leaves in two halves
unsigned m2l_half_levels(const eqfmm_plan *plan);

template <int N, typename R>
int forward_impl(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi_out,
                 void *fld_out, double *energy, int *status, unsigned char *ws, const WsLayout &W, hipStream_t st)
{
    using O = Ord<N>;
    const Geom &g = plan->g;
    const DevOps &ops = plan->ops;
    Ws<R> v = views<R>(ws, W);
    const int64_t nleaf = W.nleaf;
    const R *t = static_cast<const R *>(ops.t), *den = static_cast<const R *>(ops.inv_den);
    const R *G = static_cast<const R *>(ops.G);
    const size_t rs = sizeof(R);

    // a1/a2: validate, split, count per cell, prefix sums
    int pk = prof_begin(plan, st, EQFMM_STAGE_BIN);
    k_clear<<<blocks(nleaf + 1, 256), 256, 0, st>>>(v.hdr, v.leafcnt, v.cursor, nleaf);
    k_count<N><<<blocks(n, 256), 256, 0, st>>>(g, ops.seg64, n, pos, q, v.cnt, v.fstart, v.smask, v.leafcnt,
                                                 v.hdr);
    EQ_CHECK(hipGetLastError());
    // every prefix is clamped to the fragment capacity: a set that needs more
    // runs on in range and reports EQFMM_EWORKSPACE
    const int fcap = int(W.fcap);
    int rc = EQFMM_OK;
    if (g.continuous) {   // fragments per charge vary only in the split modes
        rc = scan(v.cnt, v.fstart, n, v.scanblk, fcap, nullptr, st);
        if (rc) return rc;
    }
    rc = scan(v.leafcnt, v.leafstart, nleaf, v.scanblk, fcap, &v.hdr->nfrag, st);
    if (rc) return rc;
    k_emit<N, R><<<blocks(n, 256), 256, 0, st>>>(g, ops.seg64, ops.seg_den64, n, pos, q, v.fstart,
                                                 v.leafstart, v.cursor, v.su, v.sv, v.sw, v.sq,
                                                 v.spar, v.sleaf, v.gslot, v.gw, v.gdw, W.fcap);
    EQ_CHECK(hipGetLastError());
    k_fill<R><<<blocks(W.fcap, 256), 256, 0, st>>>(g, v.leafstart + nleaf, pos, q, v.smask, v.spar, v.su, v.sv,
                                                   v.sw, v.sq, v.sleaf);
    EQ_CHECK(hipGetLastError());
    prof_end(plan, st, pk, EQFMM_STAGE_BIN, 0.0, double(n) * 104.0);

    // a8: near field on the side stream, concurrent with a3-a6
    hipStream_t sd = plan->side;
    if (!sd) return EQFMM_ESTATE;
    EQ_CHECK(hipEventRecord(plan->ev_bin, st));
    EQ_CHECK(hipStreamWaitEvent(sd, plan->ev_bin, 0));
    pk = prof_begin(plan, sd, EQFMM_STAGE_LEAF);
    rc = launch_p2p<R>(plan, n, W.fcap, v.leafstart, v.su, v.sv, v.sw, v.sq, v.spar, v.sleaf, v.smask, v.sphi,
                       v.snf, sd);
    if (rc) return rc;
    prof_end(plan, sd, pk, EQFMM_STAGE_LEAF, 0.0, 0.0);
    EQ_CHECK(hipEventRecord(plan->ev_near, sd));

    // a3: replacement at the finest cells
    const int L = g.L;
    pk = prof_begin(plan, st, EQFMM_STAGE_P2M);
    {
        constexpr int CPB = O::TPC >= 256 ? 1 : 256 / O::TPC;
        const int tpb = CPB * O::TPC;
        k_p2m<N, R><<<blocks(nleaf, CPB), tpb, 0, st>>>(t, den, nleaf, v.leafstart, v.su, v.sv, v.sw,
                                                        v.sq, v.phi + W.lvl[L] * O::NS);
        EQ_CHECK(hipGetLastError());
    }
    prof_end(plan, st, pk, EQFMM_STAGE_P2M, double(n) * (2.0 * O::N3 + 9.0 * N),
             double(n) * 4 * rs + double(nleaf) * O::NS * rs);

    // a4: upward pass; free space needs Phi down to level 2, periodic to 0
    const int lmin = g.periodic ? 1 : 2;
    pk = prof_begin(plan, st, EQFMM_STAGE_M2M);
    for (int l = L; l > (g.periodic ? 0 : 2); --l) {
        const int Dl = 1 << l;
        const int64_t np = int64_t(1) << (3 * (l - 1));
        k_m2m<N, R><<<dim3(unsigned(np)), O::TPC, 0, st>>>(G, Dl, v.phi + W.lvl[l] * O::NS,
                                                           v.phi + W.lvl[l - 1] * O::NS);
        EQ_CHECK(hipGetLastError());
    }
    // every interaction level again with its halo (the far-field input)
    rc = launch_m2l_pad<R>(plan, lmin, L, W.lvl.data(), W.plvl.data(), v.phi, v.phipad, st);
    if (rc) return rc;
    prof_end(plan, st, pk, EQFMM_STAGE_M2M, 0.0, 0.0);

    // a5/a6: downward pass.  The far-field products of every interaction
    // level are computed in one launch, each storing its level's local
    // vectors; the shifts then add each parent's functional into its
    // children, top down (Psi_child = Psi_parent o shift + far terms).
    if (g.periodic) {
        k_root<R><<<1, 256, 0, st>>>(static_cast<const R *>(ops.T), O::N3, R(1.0 / g.box), v.phi, v.loc);
        EQ_CHECK(hipGetLastError());
    }
    rc = launch_m2l<R>(plan, lmin, L, W.lvl.data(), W.plvl.data(), v.phipad, v.loc, v.loc2, st);
    if (rc) return rc;
    // free space: Psi vanishes at levels 0 and 1, so the shifts start at 2 -> 3.
    // A level whose far field came in two halves gets the second half added
    // as it receives its parent's functional (the top level, a parent only,
    // as it gives it).
    const unsigned hm = m2l_half_levels(plan);
    const int l0 = g.periodic ? 1 : 3;
    for (int l = l0; l <= L; ++l) {
        pk = prof_begin(plan, st, EQFMM_STAGE_L2L);
        const int64_t np = int64_t(1) << (3 * (l - 1));
        const R *p2 = l == l0 && ((hm >> (l - 1)) & 1u) ? v.loc2 + W.lvl[l - 1] * O::NS : nullptr;
        const R *c2 = (hm >> l) & 1u ? v.loc2 + W.lvl[l] * O::NS : nullptr;
        k_l2l<N, R><<<dim3(unsigned(np)), O::TPC, 0, st>>>(G, 1 << l, v.loc + W.lvl[l - 1] * O::NS, p2,
                                                           v.loc + W.lvl[l] * O::NS, c2);
        EQ_CHECK(hipGetLastError());
        prof_end(plan, st, pk, EQFMM_STAGE_L2L, 0.0, 0.0);
    }

    // a7: far field at the fragments, added to the near-field sums
    EQ_CHECK(hipStreamWaitEvent(st, plan->ev_near, 0));
    pk = prof_begin(plan, st, EQFMM_STAGE_LEAF);
    rc = launch_l2p<N, R>(plan, W.fcap, v.leafstart, t, den, v.su, v.sv, v.sw, v.spar, v.sleaf, v.smask,
                          v.loc + W.lvl[L] * O::NS, v.sphi, v.snf, v.sfld, st);
    if (rc) return rc;
    prof_end(plan, st, pk, EQFMM_STAGE_LEAF, 0.0, 0.0);

    // a9/a10: back to the charges, energy
    pk = prof_begin(plan, st, EQFMM_STAGE_GATHER);
    k_gather<R><<<dim3(unsigned(W.e_blocks)), 256, 0, st>>>(n, q, v.fstart, v.smask, v.gslot, v.gw,
                                                            v.gdw, v.sphi, v.sfld,
                                                            static_cast<R *>(phi_out),
                                                            static_cast<R *>(fld_out), v.epart);
    k_energy<<<1, 256, 0, st>>>(v.epart, W.e_blocks, energy, v.hdr, g.periodic, W.fcap, status);
    EQ_CHECK(hipGetLastError());
    prof_end(plan, st, pk, EQFMM_STAGE_GATHER, 0.0, 0.0);
    return EQFMM_OK;
}

template <typename R>
int backward_impl(eqfmm_plan *plan, int64_t n, const double *q, const double *gE, void *dEdx,
                  void *dEdq, unsigned char *ws, const WsLayout &W, hipStream_t st)
{
    Ws<R> v = views<R>(ws, W);
    const int pk = prof_begin(plan, st, EQFMM_STAGE_ADJOINT);
    if (n > 0) {
        k_adjoint<R><<<blocks(n, 256), 256, 0, st>>>(n, q, gE, v.fstart, v.smask, v.gslot, v.gw, v.gdw,
                                                     v.sphi, v.sfld, static_cast<R *>(dEdx),
                                                     static_cast<R *>(dEdq));
        EQ_CHECK(hipGetLastError());
    }
    prof_end(plan, st, pk, EQFMM_STAGE_ADJOINT, 0.0, double(n) * (40.0 + 4.0 * sizeof(R)));
    return EQFMM_OK;
}

#define EQ_ORDER_SWITCH(n, CALL)                        \
    switch (n) {                                        \
        case 2: { constexpr int N = 2; return CALL; }   \
        case 3: { constexpr int N = 3; return CALL; }   \
        case 4: { constexpr int N = 4; return CALL; }   \
        case 5: { constexpr int N = 5; return CALL; }   \
        case 6: { constexpr int N = 6; return CALL; }   \
        case 7: { constexpr int N = 7; return CALL; }   \
        default: return EQFMM_EINVAL;                   \
    }

int run_forward(eqfmm_plan *plan, int64_t n, const double *pos, const double *q, void *phi,
                void *field, double *energy, int *status, unsigned char *ws, const WsLayout &W, hipStream_t st)
{
    if (n == 0) {
        if (energy) EQ_CHECK(hipMemsetAsync(energy, 0, sizeof(double), st));
        EQ_CHECK(hipMemsetAsync(ws + W.hdr, 0, sizeof(WsHeader), st));
        if (status) EQ_CHECK(hipMemsetAsync(status, 0, sizeof(int), st));
        return EQFMM_OK;
    }
    if (plan->p.precision == EQFMM_FP64)
        EQ_ORDER_SWITCH(plan->g.n,
                        (forward_impl<N, double>(plan, n, pos, q, phi, field, energy, status, ws, W, st)))
    EQ_ORDER_SWITCH(plan->g.n, (forward_impl<N, float>(plan, n, pos, q, phi, field, energy, status, ws, W, st)))
}

int run_backward(eqfmm_plan *plan, int64_t n, const double *q, const double *gE, void *dEdx,
                 void *dEdq, unsigned char *ws, const WsLayout &W, hipStream_t st)
{
    if (plan->p.precision == EQFMM_FP64) return backward_impl<double>(plan, n, q, gE, dEdx, dEdq, ws, W, st);
    return backward_impl<float>(plan, n, q, gE, dEdx, dEdq, ws, W, st);
}

// timing hooks for the far-field launcher (m2l.hip)
int prof_begin_m2l(eqfmm_plan *plan, hipStream_t st) { return prof_begin(plan, st, EQFMM_STAGE_M2L); }
void prof_end_m2l(eqfmm_plan *plan, hipStream_t st, int k, double flops, double bytes)
{
    prof_end(plan, st, k, EQFMM_STAGE_M2L, flops, bytes);
}

}  // namespace eqfmm
