// Far field (a5): L_c += (1/side) sum_{o in IL(c)} K_o Phi_{c+o} at one level,
// the bilinear form of Eq. (14) applied as matrix products on the matrix cores.
//
// Work decomposition: every target cell with the same parity p (cell index
// mod 2 per axis) has the same interaction list, the 189 displacements o in
// [-2-p, 3-p]^3 minus the 27 adjacent ones (children of the parent's
// neighbours that are not adjacent), padded to kListLen with zero matrices.  A wave owns 32 target cells of one
// parity (the same child of 32 parents that are consecutive in Morton order,
// a 4x4x2 block) and one 32-wide block of target nodes, and runs through the
// interaction list; for each displacement the 32 source rows form the A
// operand and the matching rows of K_o the B operand of a
//   C[cell][node] += sum_k Phi_src(cell)[k] K_o[node][k]
// product.  The source-node axis k is split in two halves, one per half
// wave, so that each lane streams one contiguous half row of Phi and of K_o.
// Each displacement's product is summed in a fresh float accumulator pair
// and only then added to the running sums: the far-field terms cancel
// heavily (charges of both signs), and one float accumulation chain over
// the whole list loses about an order of magnitude of accuracy.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace eqfmm {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The interaction levels of one evaluation, handled by a single launch:
// workgroups [wg_begin[i], wg_begin[i+1]) belong to level level[i].
struct MxLevels {
    int nlev;
    int level[8], ntile[8], wg_begin[9];
    int64_t cell0[8];      // first cell of the level in the Phi / L arrays
    float inv_side[8];
    double inv_side64[8];
};

template <int N> struct MxShape {
    static constexpr int N3 = N * N * N;
    static constexpr int NS = (N3 + 15) & ~15;   // row stride of Phi / L
    static constexpr int KH = NS / 2;            // source nodes per half wave
    static constexpr int NB = (N3 + 31) / 32;    // 32-wide target node blocks
};

namespace {

__device__ __forceinline__ int compact3(int64_t m)
{
    int v = 0;
    for (int b = 0; b < 21; ++b) v |= int((m >> (3 * b)) & 1) << b;
    return v;
}

int nb_of(int n3) { return (n3 + 31) / 32; }

// compile-time loop: f(integral_constant<int, I>) for I in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace

// ------------------------------------------------------------ operand layout

// FP32: lane l (node j = l % 32, half g = l / 32) at step s supplies
// K_o[nb*32 + j][g*KH + s]; stored [oi][nb][s/4][lane][s%4] (one 16-byte
// load per lane per four steps).  BF16: eight consecutive steps per lane,
// [oi][nb][s/8][lane][s%8].
// bytes of the float layout; the bf16 mode stores the float layout (coarse
// levels) followed by the bf16 one (the two finest levels)
size_t mx_f32_bytes(const Geom &g) { return size_t(kNumOffsets) * nb_of(g.n3) * (g.ns / 2) * 64 * sizeof(float); }

size_t mx_layout_bytes(const Geom &g, int precision)
{
    if (precision == EQFMM_FP64)   // [oi][nb16][s/2][lane][s%2], KQ = ns/4 steps
        return size_t(kNumOffsets) * ((g.n3 + 15) / 16) * (g.ns / 4) * 64 * sizeof(double);
    if (precision == EQFMM_FP32) return mx_f32_bytes(g);
    return mx_f32_bytes(g) + mx_f32_bytes(g) / 2;
}

void mx_layout_fill(const Geom &g, int precision, const std::vector<double> &K, unsigned char *dst)
{
    if (precision == EQFMM_FP64) {
        // v_mfma_f64_16x16x4f64: lane l (node j = l % 16, quarter g = l / 16)
        // at step s supplies K_o[nb*16 + j][g*KQ + s]
        const int n3 = g.n3, KQ = g.ns / 4, NB = (n3 + 15) / 16;
        double *d = reinterpret_cast<double *>(dst);
        for (int oi = 0; oi < kNumOffsets; ++oi)
            for (int nb = 0; nb < NB; ++nb)
                for (int s = 0; s < KQ; ++s)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int j = nb * 16 + (lane & 15);
                        const int k = (lane >> 4) * KQ + s;
                        const double v = (j < n3 && k < n3) ? K[(size_t(oi) * n3 + j) * n3 + k] : 0.0;
                        d[((((size_t(oi) * NB + nb) * (KQ / 2) + s / 2) * 64 + lane) * 2) + s % 2] = v;
                    }
        return;
    }
    const int n3 = g.n3, KH = g.ns / 2, NB = nb_of(n3);
    for (int pass = 0; pass < (precision == EQFMM_FP32 ? 1 : 2); ++pass) {
        const int V = pass == 0 ? 4 : 8;
        unsigned char *base = pass == 0 ? dst : dst + mx_f32_bytes(g);
        for (int oi = 0; oi < kNumOffsets; ++oi)
            for (int nb = 0; nb < NB; ++nb)
                for (int s = 0; s < KH; ++s)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int j = nb * 32 + (lane & 31);
                        const int k = (lane >> 5) * KH + s;
                        const double v = (j < n3 && k < n3) ? K[(size_t(oi) * n3 + j) * n3 + k] : 0.0;
                        const size_t idx =
                            ((((size_t(oi) * NB + nb) * (KH / V) + s / V) * 64 + lane) * V) + s % V;
                        if (pass == 0) {
                            reinterpret_cast<float *>(base)[idx] = float(v);
                        } else {
                            __hip_bfloat16 b = __float2bfloat16(float(v));
                            std::memcpy(base + idx * 2, &b, 2);
                        }
                    }
    }
}

// --------------------------------------------------------------- kernels

// grid: round_up(8 * NB * ceil(ntile / 4), 8) workgroups of 4 waves; the
// workgroup id is remapped so that each of the 8 XCDs gets a contiguous
// range of (parity, node block, tile) work, i.e. mostly one parity and
// hence one set of 189 matrices in its L2.
//
// The walk over (displacement, k-chunk) steps is software pipelined: the
// operands of step s+1 are loaded into the second register stage while the
// matrix cores work on step s.  Each displacement's product goes to a fresh
// accumulator pair that is added to float running sums when the
// displacement is complete.
template <int N, bool BF16, int CH, bool PERIODIC, int NSPLIT>
__global__ void __launch_bounds__(256) k_m2l_mx(Geom g, const void *__restrict__ Kmx,
                                                const signed char *__restrict__ offs, MxLevels lv,
                                                const float *__restrict__ phi_all,
                                                const float *__restrict__ zrow,
                                                float *__restrict__ loc_all, int nwg)
{
    using S = MxShape<N>;
    constexpr int NS = S::NS, KH = S::KH, NB = S::NB;
    constexpr int NA = KH / 4;            // float4 loads of one half row
    constexpr int NCH = NA / CH;          // pipeline steps per displacement
    static_assert(NA % CH == 0, "chunking");
    static_assert(!BF16 || CH % 2 == 0, "bf16 steps take 8 sources per lane");
    const int per = gridDim.x >> 3;
    int wg = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wg >= nwg) return;
    int li = 0;
    while (li + 1 < lv.nlev && wg >= lv.wg_begin[li + 1]) ++li;
    wg -= lv.wg_begin[li];
    const int level = lv.level[li], ntile = lv.ntile[li];
    const float inv_side = lv.inv_side[li];
    const float *phi = phi_all + lv.cell0[li] * NS;
    float *loc = loc_all + lv.cell0[li] * NS;
    // a workgroup of 4 waves holds TPW = 4 / NSPLIT tiles; NSPLIT waves share
    // one tile, each running a contiguous part of the interaction list, and
    // their sums are added in a fixed order at the end
    constexpr int TPW = 4 / NSPLIT;
    const int ntg = (ntile + TPW - 1) / TPW;
    const int tg = wg % ntg, pn = wg / ntg;
    const int nb = pn % NB, p = pn / NB;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int t = tg * TPW + wv % TPW;
    const int hs = wv / TPW;
    constexpr int OPS = kListLen / NSPLIT;           // even: displacements go in pairs
    static_assert(kListLen % (2 * NSPLIT) == 0, "list padding");
    const int o_begin = hs * OPS, o_end = o_begin + OPS;
    // the interaction list of this parity, packed (ox+3) | (oy+3) << 4 | (oz+3) << 8
    __shared__ int soff[kListLen];
    if (threadIdx.x < kListLen) {
        const signed char *q = offs + (p * kListLen + threadIdx.x) * 3;
        soff[threadIdx.x] = (q[0] + 3) | ((q[1] + 3) << 4) | ((q[2] + 3) << 8);
    }
    __syncthreads();
    const bool active = t < ntile;
    const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
    const int D = 1 << level, Dp = D >> 1;
    const int64_t nparent = int64_t(Dp) * Dp * Dp;
    const int i = lane & 31, gh = lane >> 5;
    const int64_t Pm = int64_t(t) * 32 + i;
    const bool cvalid = Pm < nparent;
    const int cx = 2 * compact3(Pm) + px, cy = 2 * compact3(Pm >> 1) + py, cz = 2 * compact3(Pm >> 2) + pz;

    float4 abuf[2][CH];
    using BT = typename std::conditional<BF16, bf16x8, float4>::type;
    constexpr int NBL = BF16 ? CH / 2 : CH;   // B loads per step
    BT bbuf[2][NBL];

    // Loads of step `step` (clamped, so that the loop body is branch free and
    // the wait counts stay exact); a source outside the box (free space)
    // reads a row of zeros.
    auto issue = [&](int step, auto bc) {
        constexpr int b = decltype(bc)::value;
        step = step < o_end * NCH ? step : o_end * NCH - 1;   // prefetch past the end
        const int oidx = step / NCH, ch = step - oidx * NCH;
        const int pk = soff[oidx];
        const int ox = (pk & 15) - 3, oy = ((pk >> 4) & 15) - 3, oz = (pk >> 8) - 3;
        int sx = cx + ox, sy = cy + oy, sz = cz + oz;
        bool valid = cvalid;
        if constexpr (PERIODIC) {
            sx &= D - 1;
            sy &= D - 1;
            sz &= D - 1;
        } else {
            valid = valid && sx >= 0 && sy >= 0 && sz >= 0 && sx < D && sy < D && sz < D;
        }
        const float *row = valid ? phi + (sx + int64_t(D) * (sy + int64_t(D) * sz)) * NS : zrow;
        const float4 *ap = reinterpret_cast<const float4 *>(row + gh * KH) + ch * CH;
#pragma unroll
        for (int c = 0; c < CH; ++c) abuf[b][c] = ap[c];
        const int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
        const BT *bp = reinterpret_cast<const BT *>(Kmx) + ((size_t(oi) * NB + nb) * (NA * 4 / (BF16 ? 8 : 4)) +
                                                            ch * NBL) * 64 + lane;
#pragma unroll
        for (int c = 0; c < NBL; ++c) bbuf[b][c] = bp[c * 64];
    };

    floatx16 c0 = {}, c1 = {}, run = {};
    // one k-chunk of one displacement from register stage b
    auto compute = [&](auto bc) {
        constexpr int b = decltype(bc)::value;
        if constexpr (!BF16) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const float4 a = abuf[b][c];
                const float4 bb = bbuf[b][c];
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bb.x, c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bb.y, c1, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bb.z, c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bb.w, c1, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NBL; ++c) {
                const float4 a0 = abuf[b][2 * c], a1 = abuf[b][2 * c + 1];
                bf16x8 a;
                a[0] = __bf16(a0.x);
                a[1] = __bf16(a0.y);
                a[2] = __bf16(a0.z);
                a[3] = __bf16(a0.w);
                a[4] = __bf16(a1.x);
                a[5] = __bf16(a1.y);
                a[6] = __bf16(a1.z);
                a[7] = __bf16(a1.w);
                if (c & 1) c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bbuf[b][c], c1, 0, 0, 0);
                else c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bbuf[b][c], c0, 0, 0, 0);
            }
        }
    };

    // Two displacements (2 * NCH steps) per trip, unrolled at compile time so
    // that the register stage of every step is a constant and the body has
    // no branches; the second displacement of the last trip is a clamped
    // repeat whose sum is discarded.
    if (active) {
        issue(o_begin * NCH, std::integral_constant<int, 0>{});
        for (int op = o_begin; op < o_end; op += 2) {
            static_for<0, 2 * NCH>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr int b = j & 1;
                constexpr int ch = j % NCH;
                issue(op * NCH + j + 1, std::integral_constant<int, 1 - b>{});
                // keep the loads of the next step ahead of this step's products
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (ch == 0) {
                    c0 = floatx16{};
                    c1 = floatx16{};
                }
                compute(std::integral_constant<int, b>{});
                if constexpr (ch == NCH - 1) run += c0 + c1;
            });
        }
    }
    if constexpr (NSPLIT > 1) {
        __shared__ floatx16 red[NSPLIT - 1][TPW][64];
        if (hs > 0) red[hs - 1][wv % TPW][lane] = run;
        __syncthreads();
        if (hs > 0) return;
#pragma unroll
        for (int h = 0; h < NSPLIT - 1; ++h) run += red[h][wv % TPW][lane];
    }
    if (!active) return;

    // C[cell][node]: lane l, register r -> node j = l % 32, cell
    // ii = 4 (l / 32) + (r % 4) + 8 (r / 4)
    const int j = nb * 32 + (lane & 31);
    if (j >= S::N3) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ii = 4 * (lane >> 5) + (r & 3) + 8 * (r >> 2);
        const int64_t P2 = int64_t(t) * 32 + ii;
        if (P2 >= nparent) continue;
        const int x = 2 * compact3(P2) + px, y = 2 * compact3(P2 >> 1) + py, z = 2 * compact3(P2 >> 2) + pz;
        const int64_t c = x + int64_t(D) * (y + int64_t(D) * z);
        loc[c * NS + j] = inv_side * run[r];
    }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Double precision on the matrix cores (v_mfma_f64_16x16x4f64): a wave owns
// 16 target cells of one parity (16 parents consecutive in Morton order) and
// 16 target nodes; the source axis is split in four quarters, one per
// quarter wave.  Same pipelining as the float kernel.
template <int N, int CH, bool PERIODIC>
__global__ void __launch_bounds__(256) k_m2l_f64(Geom g, const double2 *__restrict__ Kmx,
                                                 const signed char *__restrict__ offs, MxLevels lv,
                                                 const double *__restrict__ phi_all,
                                                 const double *__restrict__ zrow,
                                                 double *__restrict__ loc_all, int nwg)
{
    constexpr int N3 = N * N * N, NS = (N3 + 15) & ~15, KQ = NS / 4, NB = (N3 + 15) / 16;
    constexpr int NA = KQ / 2;            // double2 loads of one quarter row
    constexpr int NCH = NA / CH;
    static_assert(NA % CH == 0, "chunking");
    const int per = gridDim.x >> 3;
    int wg = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wg >= nwg) return;
    int li = 0;
    while (li + 1 < lv.nlev && wg >= lv.wg_begin[li + 1]) ++li;
    wg -= lv.wg_begin[li];
    const int level = lv.level[li], ntile = lv.ntile[li];
    const double inv_side = lv.inv_side64[li];
    const double *phi = phi_all + lv.cell0[li] * NS;
    double *loc = loc_all + lv.cell0[li] * NS;
    const int ntg = (ntile + 3) >> 2;
    const int tg = wg % ntg, pn = wg / ntg;
    const int nb = pn % NB, p = pn / NB;
    const int lane = threadIdx.x & 63;
    const int t = tg * 4 + (threadIdx.x >> 6);
    __shared__ int soff[kListLen];
    if (threadIdx.x < kListLen) {
        const signed char *q = offs + (p * kListLen + threadIdx.x) * 3;
        soff[threadIdx.x] = (q[0] + 3) | ((q[1] + 3) << 4) | ((q[2] + 3) << 8);
    }
    __syncthreads();
    if (t >= ntile) return;
    const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
    const int D = 1 << level, Dp = D >> 1;
    const int64_t nparent = int64_t(Dp) * Dp * Dp;
    const int i = lane & 15, gq = lane >> 4;
    const int64_t Pm = int64_t(t) * 16 + i;
    const bool cvalid = Pm < nparent;
    const int cx = 2 * compact3(Pm) + px, cy = 2 * compact3(Pm >> 1) + py, cz = 2 * compact3(Pm >> 2) + pz;
    double2 abuf[2][CH], bbuf[2][CH];

    auto issue = [&](int step, auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int nsteps = kListLen * NCH;
        step = step < nsteps ? step : nsteps - 1;
        const int oidx = step / NCH, ch = step - oidx * NCH;
        const int pk = soff[oidx];
        const int ox = (pk & 15) - 3, oy = ((pk >> 4) & 15) - 3, oz = (pk >> 8) - 3;
        int sx = cx + ox, sy = cy + oy, sz = cz + oz;
        bool valid = cvalid;
        if constexpr (PERIODIC) {
            sx &= D - 1;
            sy &= D - 1;
            sz &= D - 1;
        } else {
            valid = valid && sx >= 0 && sy >= 0 && sz >= 0 && sx < D && sy < D && sz < D;
        }
        const double *row = valid ? phi + (sx + int64_t(D) * (sy + int64_t(D) * sz)) * NS : zrow;
        const double2 *ap = reinterpret_cast<const double2 *>(row + gq * KQ) + ch * CH;
#pragma unroll
        for (int c = 0; c < CH; ++c) abuf[b][c] = ap[c];
        const int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
        const double2 *bp = Kmx + ((size_t(oi) * NB + nb) * NA + ch * CH) * 64 + lane;
#pragma unroll
        for (int c = 0; c < CH; ++c) bbuf[b][c] = bp[c * 64];
    };

    doublex4 c0 = {}, c1 = {}, run = {};
    issue(0, std::integral_constant<int, 0>{});
    for (int op = 0; op < kListLen; op += 2) {
        static_for<0, 2 * NCH>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int b = j & 1;
            constexpr int ch = j % NCH;
            issue(op * NCH + j + 1, std::integral_constant<int, 1 - b>{});
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (ch == 0) {
                c0 = doublex4{};
                c1 = doublex4{};
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(abuf[b][c].x, bbuf[b][c].x, c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(abuf[b][c].y, bbuf[b][c].y, c1, 0, 0, 0);
            }
            if constexpr (ch == NCH - 1) run += c0 + c1;
        });
    }
    // lane l, register r -> node j = l % 16, cell ii = l / 16 + 4 r
    const int j = nb * 16 + (lane & 15);
    if (j >= N3) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ii = (lane >> 4) + 4 * r;
        const int64_t P2 = int64_t(t) * 16 + ii;
        if (P2 >= nparent) continue;
        const int x = 2 * compact3(P2) + px, y = 2 * compact3(P2 >> 1) + py, z = 2 * compact3(P2 >> 2) + pz;
        const int64_t c = x + int64_t(D) * (y + int64_t(D) * z);
        loc[c * NS + j] = inv_side * run[r];
    }
}

// --------------------------------------------------------------- launcher

int prof_begin_m2l(eqfmm_plan *plan, hipStream_t st);
void prof_end_m2l(eqfmm_plan *plan, hipStream_t st, int k, double flops, double bytes);

namespace {

// Interaction-list pairs at one level; the count factorises over the axes:
// A = number of (x, ox) with ox in [-2-p, 3-p] and the source in range (free)
// or wrapped (periodic), B = the same with |ox| <= 1; pairs = A^3 - B^3.
double il_pairs(const Geom &g, int level)
{
    const int Dl = 1 << level;
    int64_t A = 0, B = 0;
    for (int x = 0; x < Dl; ++x)
        for (int ox = -2 - (x & 1); ox <= 3 - (x & 1); ++ox) {
            if (!g.periodic && (x + ox < 0 || x + ox >= Dl)) continue;
            ++A;
            if (ox >= -1 && ox <= 1) ++B;
        }
    return double(A) * A * A - double(B) * B * B;
}

// Level table: tiles of `cells_per_tile` parents per (parity, node block),
// `tpw` tiles per workgroup.
int fill_levels(const Geom &g, int lmin, int lmax, const int64_t *lvl, int cells_per_tile, int nb, int tpw,
                MxLevels &lv)
{
    lv.nlev = lmax - lmin + 1;
    int wgs = 0;
    for (int i = 0; i < lv.nlev; ++i) {
        const int l = lmin + i;
        const int Dp = (1 << l) >> 1;
        const int64_t nparent = int64_t(Dp) * Dp * Dp;
        lv.level[i] = l;
        lv.ntile[i] = int((nparent + cells_per_tile - 1) / cells_per_tile);
        lv.wg_begin[i] = wgs;
        wgs += 8 * nb * ((lv.ntile[i] + tpw - 1) / tpw);
        lv.cell0[i] = lvl[l];
        lv.inv_side[i] = float(double(1 << l) / g.box);
        lv.inv_side64[i] = double(1 << l) / g.box;
    }
    lv.wg_begin[lv.nlev] = wgs;
    return wgs;
}

// k-chunk per pipeline step (float4 loads of A and of B per lane): 4 for
// n <= 4, where more resident waves pay off, 8 above (measured)
template <int N> struct MxChunk {
    static constexpr int NA = MxShape<N>::KH / 4;
    static constexpr int CH = N <= 4 ? (NA % 4 == 0 ? 4 : NA) : (NA % 8 == 0 ? 8 : (NA % 4 == 0 ? 4 : NA));
};

template <int N>
int launch_mx(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const float *phi, const float *zrow,
              float *loc, hipStream_t st)
{
    using S = MxShape<N>;
    constexpr int CH = MxChunk<N>::CH;
    const Geom &g = plan->g;
    const signed char *offs = static_cast<const signed char *>(plan->ops.offs);
    // waves per tile: enough waves to keep every SIMD busy
    int64_t tiles = 0;
    for (int l = lmin; l <= lmax; ++l) {
        const int64_t Dp = (int64_t(1) << l) >> 1;
        tiles += 8 * S::NB * ((Dp * Dp * Dp + 31) / 32);
    }
    const int split = tiles >= 4096 ? 1 : (tiles >= 1024 ? 2 : 4);
    // bf16 inputs only on the two finest levels, which carry nearly all the
    // work; on coarse levels the cells hold many charges and bf16 rounding of
    // their large, sign-cancelling vectors leaves a spurious net charge
    const bool bf = plan->p.precision == EQFMM_FP32_BF16FAR;
    const void *Kbf = static_cast<const unsigned char *>(plan->ops.Kmx) + mx_f32_bytes(g);
    auto go = [&](int l0, int l1, bool use_bf) -> int {
        if (l0 > l1) return EQFMM_OK;
        MxLevels lv;
        const int nwg = fill_levels(g, l0, l1, lvl, 32, S::NB, 4 / split, lv);
        const int grid = (nwg + 7) & ~7;
        const void *K = use_bf ? Kbf : plan->ops.Kmx;
#define EQ_M2L_LAUNCH(B, P, SP) \
    k_m2l_mx<N, B, CH, P, SP><<<grid, 256, 0, st>>>(g, K, offs, lv, phi, zrow, loc, nwg)
#define EQ_M2L_SPLIT(B, P)                           \
    if (split == 1) EQ_M2L_LAUNCH(B, P, 1);          \
    else if (split == 2) EQ_M2L_LAUNCH(B, P, 2);     \
    else EQ_M2L_LAUNCH(B, P, 4);
        if (use_bf && g.periodic) { EQ_M2L_SPLIT(true, true) }
        else if (use_bf) { EQ_M2L_SPLIT(true, false) }
        else if (g.periodic) { EQ_M2L_SPLIT(false, true) }
        else { EQ_M2L_SPLIT(false, false) }
#undef EQ_M2L_SPLIT
#undef EQ_M2L_LAUNCH
        return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
    };
    if (!bf) return go(lmin, lmax, false);
    const int lb = lmax - 1 > lmin ? lmax - 1 : lmin;
    const int rc = go(lmin, lb - 1, false);
    return rc ? rc : go(lb, lmax, true);
}

template <int N>
int launch_f64(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const double *phi, const double *zrow,
               double *loc, hipStream_t st)
{
    constexpr int NA = ((N * N * N + 15) & ~15) / 8;
    constexpr int CH = NA % 4 == 0 ? 4 : (NA % 2 == 0 ? 2 : 1);
    constexpr int NB = (N * N * N + 15) / 16;
    const Geom &g = plan->g;
    MxLevels lv;
    const int nwg = fill_levels(g, lmin, lmax, lvl, 16, NB, 4, lv);
    const int grid = (nwg + 7) & ~7;
    const double2 *K = static_cast<const double2 *>(plan->ops.Kmx);
    const signed char *offs = static_cast<const signed char *>(plan->ops.offs);
    if (g.periodic)
        k_m2l_f64<N, CH, true><<<grid, 256, 0, st>>>(g, K, offs, lv, phi, zrow, loc, nwg);
    else
        k_m2l_f64<N, CH, false><<<grid, 256, 0, st>>>(g, K, offs, lv, phi, zrow, loc, nwg);
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

}  // namespace

// All interaction levels lmin..lmax in one launch (two for the bf16 mode);
// each writes (stores) its level's local vectors.
template <typename R>
int launch_m2l(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const R *phi, const R *zrow, R *loc,
               hipStream_t st)
{
    const Geom &g = plan->g;
    const int pk = prof_begin_m2l(plan, st);
    int rc = EQFMM_EINVAL;
#define EQ_CASE(NN)                                                                          \
    case NN:                                                                                 \
        if constexpr (sizeof(R) == sizeof(float))                                            \
            rc = launch_mx<NN>(plan, lmin, lmax, lvl, phi, zrow, loc, st);                   \
        else                                                                                 \
            rc = launch_f64<NN>(plan, lmin, lmax, lvl, phi, zrow, loc, st);                  \
        break;
    switch (g.n) {
        EQ_CASE(2) EQ_CASE(3) EQ_CASE(4) EQ_CASE(5) EQ_CASE(6) EQ_CASE(7)
        default: break;
    }
#undef EQ_CASE
    double flops = 0.0, bytes = 0.0;
    for (int l = lmin; l <= lmax; ++l) {
        flops += 2.0 * double(g.n3) * g.n3 * il_pairs(g, l);
        bytes += double(int64_t(1) << (3 * l)) * g.ns * sizeof(R) * 2.0;
    }
    prof_end_m2l(plan, st, pk, flops, bytes);
    return rc;
}

template int launch_m2l<float>(eqfmm_plan *, int, int, const int64_t *, const float *, const float *, float *,
                               hipStream_t);
template int launch_m2l<double>(eqfmm_plan *, int, int, const int64_t *, const double *, const double *,
                                double *, hipStream_t);

}  // namespace eqfmm
