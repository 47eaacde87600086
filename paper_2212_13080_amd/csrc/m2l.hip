// Far field (a5): L_c += (1/side) sum_{o in IL(c)} K_o Phi_{c+o} at one level,
// the bilinear form of Eq. (14) applied as matrix products on the matrix cores.
//
// Work decomposition: every target cell with the same parity p (cell index
// mod 2 per axis) has the same interaction list, the 189 displacements o in
// [-2-p, 3-p]^3 minus the 27 adjacent ones (children of the parent's
// neighbours that are not adjacent).  A wave owns 32 target cells of one
// parity (the same child of 32 parents that are consecutive in Morton order,
// a 4x4x2 block) and one 32-wide block of target nodes, and runs through the
// interaction list; for each displacement the 32 source rows form the A
// operand and the matching rows of K_o the B operand of a
//   C[cell][node] += sum_k Phi_src(cell)[k] K_o[node][k]
// product.  The source-node axis k is split in two halves, one per half
// wave, so that each lane streams one contiguous half row of Phi and of K_o.
// Each displacement's product is summed in a fresh float accumulator and
// folded into double sums: the far-field terms cancel heavily (charges of
// both signs), and plain float accumulation over the whole list would lose
// about an order of magnitude of accuracy.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstring>

#include "internal.h"

namespace eqfmm {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

}  // namespace

// ------------------------------------------------------------ operand layout

// FP32: lane l (node j = l % 32, half g = l / 32) at step s supplies
// K_o[nb*32 + j][g*KH + s]; stored [oi][nb][s/4][lane][s%4] (one 16-byte
// load per lane per four steps).  BF16: eight consecutive steps per lane,
// [oi][nb][s/8][lane][s%8].
size_t mx_layout_bytes(const Geom &g, int precision)
{
    if (precision == EQFMM_FP64) return 0;
    const size_t elem = precision == EQFMM_FP32 ? sizeof(float) : sizeof(__hip_bfloat16);
    return size_t(kNumOffsets) * nb_of(g.n3) * (g.ns / 2) * 64 * elem;
}

void mx_layout_fill(const Geom &g, int precision, const std::vector<double> &K, unsigned char *dst)
{
    if (precision == EQFMM_FP64) return;
    const int n3 = g.n3, KH = g.ns / 2, NB = nb_of(n3);
    const int V = precision == EQFMM_FP32 ? 4 : 8;
    for (int oi = 0; oi < kNumOffsets; ++oi)
        for (int nb = 0; nb < NB; ++nb)
            for (int s = 0; s < KH; ++s)
                for (int lane = 0; lane < 64; ++lane) {
                    const int j = nb * 32 + (lane & 31);
                    const int k = (lane >> 5) * KH + s;
                    const double v = (j < n3 && k < n3) ? K[(size_t(oi) * n3 + j) * n3 + k] : 0.0;
                    const size_t idx = ((((size_t(oi) * NB + nb) * (KH / V) + s / V) * 64 + lane) * V) + s % V;
                    if (precision == EQFMM_FP32) {
                        reinterpret_cast<float *>(dst)[idx] = float(v);
                    } else {
                        __hip_bfloat16 b = __float2bfloat16(float(v));
                        std::memcpy(dst + idx * 2, &b, 2);
                    }
                }
}

// --------------------------------------------------------------- kernels

// grid: round_up(8 * NB * ceil(ntile / 4), 8) workgroups of 4 waves; the
// workgroup id is remapped so that each of the 8 XCDs gets a contiguous
// range of (parity, node block, tile) work, i.e. mostly one parity and
// hence one set of 189 matrices in its L2.
template <int N, bool BF16>
__global__ void __launch_bounds__(256) k_m2l_mx(Geom g, const void *__restrict__ Kmx, int level,
                                                float inv_side, const float *__restrict__ phi,
                                                float *__restrict__ loc, int ntile, int nwg)
{
    using S = MxShape<N>;
    constexpr int NS = S::NS, KH = S::KH, NB = S::NB;
    const int per = gridDim.x >> 3;
    const int wg = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wg >= nwg) return;
    const int ntg = (ntile + 3) >> 2;
    const int tg = wg % ntg, pn = wg / ntg;
    const int nb = pn % NB, p = pn / NB;
    const int lane = threadIdx.x & 63;
    const int t = tg * 4 + (threadIdx.x >> 6);
    if (t >= ntile) return;
    const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
    const int D = 1 << level, Dp = D >> 1;
    const int64_t nparent = int64_t(Dp) * Dp * Dp;
    // A-operand row: cell i = lane % 32 of this tile, source half gh
    const int i = lane & 31, gh = lane >> 5;
    const int64_t Pm = int64_t(t) * 32 + i;
    const bool cvalid = Pm < nparent;
    const int cx = 2 * compact3(Pm) + px, cy = 2 * compact3(Pm >> 1) + py, cz = 2 * compact3(Pm >> 2) + pz;

    double sum[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[r] = 0.0;

    for (int oz = -2 - pz; oz <= 3 - pz; ++oz)
        for (int oy = -2 - py; oy <= 3 - py; ++oy)
            for (int ox = -2 - px; ox <= 3 - px; ++ox) {
                if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) continue;
                int sx = cx + ox, sy = cy + oy, sz = cz + oz;
                bool valid = cvalid;
                if (g.periodic) {
                    sx &= D - 1;
                    sy &= D - 1;
                    sz &= D - 1;
                } else {
                    valid = valid && sx >= 0 && sy >= 0 && sz >= 0 && sx < D && sy < D && sz < D;
                }
                if (__ballot(valid) == 0) continue;
                const int64_t src = valid ? sx + int64_t(D) * (sy + int64_t(D) * sz) : 0;
                const float *ap = phi + src * NS + gh * KH;
                const int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
                floatx16 c0 = {}, c1 = {};
                if constexpr (!BF16) {
                    const float4 *bp = reinterpret_cast<const float4 *>(Kmx) +
                                       (size_t(oi) * NB + nb) * (KH / 4) * 64 + lane;
#pragma unroll
                    for (int s4 = 0; s4 < KH / 4; ++s4) {
                        float4 a = *reinterpret_cast<const float4 *>(ap + 4 * s4);
                        const float4 b = bp[s4 * 64];
                        if (!valid) a = make_float4(0.f, 0.f, 0.f, 0.f);
                        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, c0, 0, 0, 0);
                        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, c1, 0, 0, 0);
                        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, c0, 0, 0, 0);
                        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, c1, 0, 0, 0);
                    }
                } else {
                    const bf16x8 *bp = reinterpret_cast<const bf16x8 *>(Kmx) +
                                       (size_t(oi) * NB + nb) * (KH / 8) * 64 + lane;
#pragma unroll
                    for (int s8 = 0; s8 < KH / 8; ++s8) {
                        const float4 a0 = *reinterpret_cast<const float4 *>(ap + 8 * s8);
                        const float4 a1 = *reinterpret_cast<const float4 *>(ap + 8 * s8 + 4);
                        const bf16x8 b = bp[s8 * 64];
                        const float m = valid ? 1.f : 0.f;
                        bf16x8 a;
                        a[0] = __bf16(a0.x * m);
                        a[1] = __bf16(a0.y * m);
                        a[2] = __bf16(a0.z * m);
                        a[3] = __bf16(a0.w * m);
                        a[4] = __bf16(a1.x * m);
                        a[5] = __bf16(a1.y * m);
                        a[6] = __bf16(a1.z * m);
                        a[7] = __bf16(a1.w * m);
                        if (s8 & 1) c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
                        else c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) sum[r] += double(c0[r]) + double(c1[r]);
            }

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
        loc[c * NS + j] += inv_side * float(sum[r]);
    }
}

// Plain double-precision kernel: one thread per (cell, node).
template <typename R>
__global__ void __launch_bounds__(256) k_m2l_valu(Geom g, const R *K, int Dl, R inv_side,
                                                  const R *phi, R *loc)
{
    const int n3 = g.n3, ns = g.ns;
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t c = gid / ns;
    const int a = int(gid % ns);
    const int64_t ncell = int64_t(Dl) * Dl * Dl;
    if (c >= ncell || a >= n3) return;
    const int x = int(c % Dl), y = int((c / Dl) % Dl), z = int(c / (int64_t(Dl) * Dl));
    const int px = x & 1, py = y & 1, pz = z & 1;
    R acc = R(0);
    for (int oz = -2 - pz; oz <= 3 - pz; ++oz)
        for (int oy = -2 - py; oy <= 3 - py; ++oy)
            for (int ox = -2 - px; ox <= 3 - px; ++ox) {
                if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) continue;
                int sx = x + ox, sy = y + oy, sz = z + oz;
                if (g.periodic) {
                    sx = (sx + 4 * Dl) % Dl;
                    sy = (sy + 4 * Dl) % Dl;
                    sz = (sz + 4 * Dl) % Dl;
                } else if (sx < 0 || sy < 0 || sz < 0 || sx >= Dl || sy >= Dl || sz >= Dl) {
                    continue;
                }
                const int64_t src = sx + int64_t(Dl) * (sy + int64_t(Dl) * sz);
                const int oi = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
                const R *Kr = K + (int64_t(oi) * n3 + a) * n3;
                const R *ps = phi + src * ns;
                for (int b = 0; b < n3; ++b) acc += Kr[b] * ps[b];
            }
    loc[c * ns + a] += inv_side * acc;
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

template <int N>
int launch_mx(eqfmm_plan *plan, int level, const float *phi_l, float *loc_l, hipStream_t st)
{
    using S = MxShape<N>;
    const Geom &g = plan->g;
    const int Dp = (1 << level) >> 1;
    const int64_t nparent = int64_t(Dp) * Dp * Dp;
    const int ntile = int((nparent + 31) / 32);
    const int nwg = 8 * S::NB * ((ntile + 3) / 4);
    const int grid = (nwg + 7) & ~7;
    const float inv_side = float(double(1 << level) / g.box);
    if (plan->p.precision == EQFMM_FP32_BF16FAR)
        k_m2l_mx<N, true><<<grid, 256, 0, st>>>(g, plan->ops.Kmx, level, inv_side, phi_l, loc_l, ntile, nwg);
    else
        k_m2l_mx<N, false><<<grid, 256, 0, st>>>(g, plan->ops.Kmx, level, inv_side, phi_l, loc_l, ntile, nwg);
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

}  // namespace

template <typename R>
int launch_m2l(eqfmm_plan *plan, int level, const R *phi_l, R *loc_l, hipStream_t st);

template <>
int launch_m2l<float>(eqfmm_plan *plan, int level, const float *phi_l, float *loc_l, hipStream_t st)
{
    const Geom &g = plan->g;
    const int pk = prof_begin_m2l(plan, st);
    int rc;
    switch (g.n) {
        case 2: rc = launch_mx<2>(plan, level, phi_l, loc_l, st); break;
        case 3: rc = launch_mx<3>(plan, level, phi_l, loc_l, st); break;
        case 4: rc = launch_mx<4>(plan, level, phi_l, loc_l, st); break;
        case 5: rc = launch_mx<5>(plan, level, phi_l, loc_l, st); break;
        case 6: rc = launch_mx<6>(plan, level, phi_l, loc_l, st); break;
        case 7: rc = launch_mx<7>(plan, level, phi_l, loc_l, st); break;
        default: rc = EQFMM_EINVAL;
    }
    const int64_t ncell = int64_t(1) << (3 * level);
    prof_end_m2l(plan, st, pk, 2.0 * double(g.n3) * g.n3 * il_pairs(g, level),
                 double(ncell) * g.ns * sizeof(float) * 3.0);
    return rc;
}

template <>
int launch_m2l<double>(eqfmm_plan *plan, int level, const double *phi_l, double *loc_l, hipStream_t st)
{
    const Geom &g = plan->g;
    const int Dl = 1 << level;
    const int64_t ncell = int64_t(Dl) * Dl * Dl;
    const int pk = prof_begin_m2l(plan, st);
    const int64_t work = ncell * g.ns;
    k_m2l_valu<double><<<unsigned((work + 255) / 256), 256, 0, st>>>(
        g, static_cast<const double *>(plan->ops.K), Dl, double(Dl) / g.box, phi_l, loc_l);
    const int rc = hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
    prof_end_m2l(plan, st, pk, 2.0 * double(g.n3) * g.n3 * il_pairs(g, level),
                 double(ncell) * g.ns * sizeof(double) * 3.0);
    return rc;
}

}  // namespace eqfmm
