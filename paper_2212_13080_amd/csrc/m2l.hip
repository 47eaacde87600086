// Far field (a5): L_c += (1/side) sum_{o in IL(c)} K_o Phi_{c+o} at one level,
// the bilinear form of Eq. (14) applied as matrix products on the matrix cores.
//
// Work decomposition: every target cell with the same parity p (cell index
// mod 2 per axis) has the same interaction list, the 189 displacements o in
// [-2-p, 3-p]^3 minus the 27 adjacent ones (children of the parent's
// neighbours that are not adjacent), padded to kListLen with zero matrices.
// A wave owns 32 target cells of one parity (the same child of 32 parents
// that are consecutive in Morton order, a 4x4x2 block) and one 32-wide block
// of target nodes, and runs through the interaction list; for each
// displacement the 32 source rows form the A operand and the matching rows
// of K_o the B operand of a
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
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Levels of one far-field launch, finest first.  Each XCD (blockIdx % 8)
// takes a contiguous share of every level's workgroups, the finest level's
// first; a level marked `half` splits every list between two workgroups, the
// second storing into the second L buffer.
struct MxLevels {
    int nlev;
    int level[8], ntile[8], nwg[8], share[8], rbeg[9], half[8];
    int64_t cell0[8];      // first cell of the level in the L array
    int64_t pcell0[8];     // first cell of the level in the haloed Phi
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

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
constexpr int lcm_c(int a, int b) { return a / gcd_c(a, b) * b; }

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

// ------------------------------------------------------------- halo copy

// Levels of one halo-copy launch: rows [row0[i], row0[i+1]) belong to level
// level[i], read from cell src0[i] of Phi and written from cell dst0[i] of
// the haloed copy.
struct MxPad {
    int nlev;
    int level[10];
    int64_t row0[11];
    int64_t src0[10], dst0[10];
};

// Phi of the interaction levels in the haloed layout: level l becomes a cube
// of side P = 2^l + 2 kHalo whose cell (x, y, z), counted from -kHalo, holds
// Phi_{x,y,z} inside the box, the periodic image in the periodic modes and
// zero in free space outside it.  One thread per 16 bytes of a row.
template <typename V, int VPR>
__global__ void __launch_bounds__(256) k_m2l_pad(MxPad pd, int periodic, const V *__restrict__ phi,
                                                 V *__restrict__ pad)
{
    const int64_t gid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t row = gid / VPR;
    const int e = int(gid - row * VPR);
    if (row >= pd.row0[pd.nlev]) return;
    int li = 0;
    while (li + 1 < pd.nlev && row >= pd.row0[li + 1]) ++li;
    const int r = int(row - pd.row0[li]);
    const int D = 1 << pd.level[li], P = D + 2 * kHalo;
    const int x = r % P - kHalo, y = (r / P) % P - kHalo, z = r / (P * P) - kHalo;
    V v = {};
    if (periodic || (x >= 0 && y >= 0 && z >= 0 && x < D && y < D && z < D)) {
        const int64_t c = (x & (D - 1)) + int64_t(D) * ((y & (D - 1)) + int64_t(D) * (z & (D - 1)));
        v = phi[(pd.src0[li] + c) * VPR + e];
    }
    pad[(pd.dst0[li] + r) * VPR + e] = v;
}

// --------------------------------------------------------------- kernels

// ------------------------------------------------- LDS-staged float kernel

// 16 bytes per lane from global memory straight into LDS: lane l's bytes land
// at LDS byte address lds + 16 l (lds wave-uniform, passed in M0).  Written
// as inline assembly because the compiler, for its own LDS-DMA builtin,
// waits for every copy in flight before any LDS read, which would undo the
// ring; here the kernel waits on vmcnt itself.  M0 is a reserved register:
// the far-field kernels hold no value of their own in it (every M0 write in
// their code comes from this block), so overwriting it is safe.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const void *gptr, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(gptr), "s"(lds)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// wait until at most V vector-memory operations of this wave are in flight
template <int V> __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(V >= 0 && V < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((V & 15) | ((V >> 4) << 14) | (7 << 4) | (15 << 8));
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ void wait_lgkm0()
{
    __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ void wg_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Position of 16-byte piece c of lane q's row chunk among the CH pieces of
// that lane in LDS: rotated so that the 64 lanes' reads of one piece index
// fall on distinct banks (checked for 64 banks x 16 lanes and 32 banks x 8
// lanes per pass).
template <int CH> __device__ __forceinline__ int lds_rot(int q)
{
    if constexpr (CH == 1) return 0;
    else if constexpr (CH == 2) return (q >> 2) + (q >> 3);
    else if constexpr (CH == 4) return q + (q >> 2);
    else return q + (q >> 3);
}

// The float and bf16 contraction, with the operands staged through LDS.
//
// A workgroup holds TPW = 4 / NSPLIT tiles of one (parity, node block) and
// NSPLIT parts of the interaction list.  Per step every wave copies its
// tile's chunk of source rows into LDS, 16 bytes per lane with consecutive
// lanes on consecutive bytes of a row (coalesced), and the TPW waves of a
// list part share one copy of the matrix chunk.  The copies go straight from
// global memory to LDS into a ring of NST stages, NST - 1 steps ahead of the
// products, so that reads that miss L2 are covered without holding them in
// registers; one barrier per step publishes a stage and retires the oldest.
//
// Workgroups are numbered (tile group, parity, node block) with the node
// block fastest, level by level, and the id is remapped so that each of the
// 8 XCDs gets a contiguous range: a compact region of space whose targets of
// all parities share their sources in that XCD's L2.
// Element and tile shapes of the three forms: float and bf16 products use
// v_mfma_f32_32x32x2f32 / v_mfma_f32_32x32x16_bf16 on 32 target cells x 32
// nodes with the source axis in two halves; double uses v_mfma_f64_16x16x4f64
// on 16 cells x 16 nodes with the source axis in four quarters.
enum { MX_F32 = 0, MX_BF16 = 1, MX_F64 = 2 };
template <int N, int MODE> struct MxForm {
    static constexpr bool F64 = MODE == MX_F64, BF16 = MODE == MX_BF16;
    using E = typename std::conditional<F64, double, float>::type;      // Phi, L
    using BT = typename std::conditional<F64, double2,
                                         typename std::conditional<BF16, bf16x8, float4>::type>::type;
    using ACC = typename std::conditional<F64, doublex4, floatx16>::type;
    static constexpr int N3 = N * N * N, NS = (N3 + 15) & ~15;
    static constexpr int CELLS = F64 ? 16 : 32;     // target cells (parents) per tile
    static constexpr int KG = F64 ? 4 : 2;          // source-axis groups (lane groups)
    static constexpr int KP = NS / KG;              // sources per group
    static constexpr int EPP = 16 / int(sizeof(E)); // elements per 16-byte piece
    static constexpr int NA = KP / EPP;             // pieces per group of one row
    static constexpr int NB = (N3 + CELLS - 1) / CELLS;   // node blocks
    static constexpr int REGS = F64 ? 4 : 16;       // accumulator registers
};

template <int N, int MODE, int CH, int NSPLIT, int NST>
__global__ void __launch_bounds__(256) k_m2l_lds(const void *__restrict__ Kmx, const int *__restrict__ mxtab,
                                                 MxLevels lv, const void *__restrict__ phipad_,
                                                 void *__restrict__ loc_all_, void *__restrict__ loc2_all_)
{
    using F = MxForm<N, MODE>;
    using E = typename F::E;
    using BT = typename F::BT;
    using ACC = typename F::ACC;
    constexpr bool BF16 = F::BF16, F64 = F::F64;
    constexpr int NS = F::NS, KP = F::KP, NB = F::NB, NA = F::NA, CELLS = F::CELLS, EPP = F::EPP;
    constexpr int NCH = NA / CH;          // steps per displacement
    static_assert(NA % CH == 0 && (CH & (CH - 1)) == 0 && CH <= 8, "chunking");
    static_assert(!BF16 || CH % 2 == 0, "bf16 steps take 8 sources per lane");
    static_assert(NST >= 2, "ring depth");
    constexpr int NBL = BF16 ? CH / 2 : CH;   // matrix pieces per lane and step
    constexpr int NBK = BF16 ? NA / 2 : NA;   // matrix pieces per lane, node block and displacement
    constexpr int TPW = 4 / NSPLIT;
    constexpr int BPW = (NBL + TPW - 1) / TPW;   // matrix copies per wave and step
    constexpr int DPS = CH + BPW;                // copies per wave and step
    constexpr int AU = 64 * CH, BU = 64 * NBL, SU = 4 * AU + NSPLIT * BU;   // 16-byte units
    __shared__ float4 ring[NST * SU];
    __shared__ int stab[kListLen];
    const E *phipad = static_cast<const E *>(phipad_);
    E *loc_all = static_cast<E *>(loc_all_);

    const int rr = blockIdx.x >> 3;
    int li = 0;
    while (li + 1 < lv.nlev && rr >= lv.rbeg[li + 1]) ++li;
    int wg = (blockIdx.x & 7) * lv.share[li] + (rr - lv.rbeg[li]);
    if (wg >= lv.nwg[li]) return;
    const int hv = lv.half[li], h = wg & hv;
    wg >>= hv;
    const int level = lv.level[li], ntile = lv.ntile[li];
    const E inv_side = F64 ? E(lv.inv_side64[li]) : E(lv.inv_side[li]);
    E *loc = (h ? static_cast<E *>(loc2_all_) : loc_all) + lv.cell0[li] * NS;
    // workgroups (tile group, parity, node block), node block fastest
    const int nb = wg % NB, tp = wg / NB;
    const int p = tp & 7, tg = tp >> 3;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tw = wv % TPW, hs = wv / TPW;
    const int t = tg * TPW + tw;
    const bool active = t < ntile;
    const int ta = active ? t : tg * TPW;   // idle waves copy a valid tile (and store nothing)
    // list part of this wave: NSPLIT parts per workgroup, twice as many (and
    // half as long) on a level whose lists two workgroups share
    const int ops = kListLen / (NSPLIT << hv);
    const int o_begin = (h * NSPLIT + hs) * ops, o_end = o_begin + ops;
    if (threadIdx.x < kListLen) stab[threadIdx.x] = mxtab[(level * 8 + p) * kListLen + threadIdx.x];
    __syncthreads();

    const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
    const int D = 1 << level, Dp = D >> 1, P = D + 2 * kHalo;
    const int64_t nparent = int64_t(Dp) * Dp * Dp;
    const int64_t Pm0 = int64_t(ta) * CELLS;
    const int x0 = 2 * compact3(Pm0) + px, y0 = 2 * compact3(Pm0 >> 1) + py, z0 = 2 * compact3(Pm0 >> 2) + pz;
    const E *phi0 =
        phipad + (lv.pcell0[li] + (int64_t(z0 + kHalo) * P + (y0 + kHalo)) * P + (x0 + kHalo)) * NS;
    // source-row copies: copy m, lane l fills unit u = 64 m + l of the wave's
    // chunk, i.e. piece c of consumer lane q = u / CH (cell q % CELLS,
    // source group q / CELLS)
    uint32_t voffA[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
        const int u = 64 * m + lane, q = u / CH;
        const int c = ((u % CH) - lds_rot<CH>(q)) & (CH - 1);
        const int64_t Pq = Pm0 + (q % CELLS);
        const int64_t Pl = Pq < nparent ? Pq : Pm0;
        const int cx = 2 * compact3(Pl) + px, cy = 2 * compact3(Pl >> 1) + py, cz = 2 * compact3(Pl >> 2) + pz;
        voffA[m] = uint32_t(((((cz - z0) * P + (cy - y0)) * P + (cx - x0)) * NS + (q / CELLS) * KP + EPP * c) *
                            int(sizeof(E)));
    }
    // LDS addresses (bytes) of the ring, and this lane's read offsets
    const uint32_t ring_lds = uint32_t(reinterpret_cast<uintptr_t>(ring));
    const char *kb = static_cast<const char *>(Kmx) + size_t(nb) * NBK * 64 * sizeof(BT);

    // the copies of one step: wave-uniform source bases and LDS destinations
    struct Copy {
        const char *ab, *bb;
        uint32_t la, lb;
    };
    auto setup = [&](int step, auto bc) {
        constexpr int b = decltype(bc)::value;
        step = step < o_end * NCH ? step : o_end * NCH - 1;   // copies past the end land unused
        const int oidx = step / NCH, ch = step - oidx * NCH;
        const int e = __builtin_amdgcn_readfirstlane(stab[oidx]);
        const int oi = e & 511, delta = e >> 9;
        Copy cp;
        cp.ab = reinterpret_cast<const char *>(phi0 + int64_t(delta) * NS + ch * CH * EPP);
        cp.la = ring_lds + uint32_t((b * SU + wv * AU) * 16);
        cp.bb = kb + (size_t(oi) * NB * NBK + size_t(ch) * NBL) * 64 * sizeof(BT);
        cp.lb = ring_lds + uint32_t((b * SU + 4 * AU + hs * BU) * 16);
        return cp;
    };
    auto copy_a = [&](const Copy &cp, int m) { lds_dma16(cp.ab + voffA[m], cp.la + m * 1024); };
    auto copy_b = [&](const Copy &cp, int k) {
        int j = tw + k * TPW;
        j = j < NBL ? j : NBL - 1;   // surplus copies repeat the last piece
        lds_dma16(cp.bb + (size_t(j) * 64 + lane) * sizeof(BT), cp.lb + j * 1024);
    };
    auto issue = [&](int step, auto bc) {
        const Copy cp = setup(step, bc);
#pragma unroll
        for (int m = 0; m < CH; ++m) copy_a(cp, m);
#pragma unroll
        for (int k = 0; k < BPW; ++k) copy_b(cp, k);
    };

    float4 abuf[2][CH];   // 16-byte pieces (four floats or two doubles)
    BT bbuf[2][NBL];
    auto read = [&](auto bc, auto rc) {
        constexpr int b = decltype(bc)::value, r = decltype(rc)::value;
        const float4 *ra = ring + b * SU + wv * AU + lane * CH;
        const int rot = lds_rot<CH>(lane);
#pragma unroll
        for (int c = 0; c < CH; ++c) abuf[r][c] = ra[(c + rot) & (CH - 1)];
        const float4 *rb = ring + b * SU + 4 * AU + hs * BU + lane;
#pragma unroll
        for (int j = 0; j < NBL; ++j) {
            const float4 v = rb[j * 64];
            __builtin_memcpy(&bbuf[r][j], &v, 16);
        }
    };

    ACC ca0 = {}, ca1 = {}, cb0 = {}, cb1 = {}, run = {};
    // the products of 16-byte piece c (float, double) or pair of pieces
    // (bf16) of register set r into (x0, x1)
    auto product = [&](auto rc, int c, ACC &x0, ACC &x1) {
        constexpr int r = decltype(rc)::value;
        if constexpr (F64) {
            double2 a, bv;
            __builtin_memcpy(&a, &abuf[r][c], 16);
            bv = bbuf[r][c];
            x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bv.x, x0, 0, 0, 0);
            x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bv.y, x1, 0, 0, 0);
        } else if constexpr (!BF16) {
            const float4 a = abuf[r][c];
            const float4 bv = bbuf[r][c];
            x0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bv.x, x0, 0, 0, 0);
            x1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bv.y, x1, 0, 0, 0);
            x0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bv.z, x0, 0, 0, 0);
            x1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bv.w, x1, 0, 0, 0);
        } else {
            const float4 a0 = abuf[r][2 * c], a1 = abuf[r][2 * c + 1];
            bf16x8 a;
            a[0] = __bf16(a0.x);
            a[1] = __bf16(a0.y);
            a[2] = __bf16(a0.z);
            a[3] = __bf16(a0.w);
            a[4] = __bf16(a1.x);
            a[5] = __bf16(a1.y);
            a[6] = __bf16(a1.z);
            a[7] = __bf16(a1.w);
            if (c & 1) x1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bbuf[r][c], x1, 0, 0, 0);
            else x0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bbuf[r][c], x0, 0, 0, 0);
        }
    };
    constexpr int NPR = BF16 ? NBL : CH;   // product groups per step
    // Trip of TS steps: a multiple of NST (ring stage), of 2 (register set)
    // and of 2 NCH (an even number of displacements, for the alternating
    // accumulator pairs), unrolled so that all three are constants.
    constexpr int TS = lcm_c(lcm_c(NST, 2), 2 * NCH), TD = TS / NCH;
    static_assert((kListLen / NSPLIT) % TD == 0 && (kListLen / (2 * NSPLIT)) % TD == 0, "pipeline trip");
    const int s0 = o_begin * NCH;
    static_for<0, NST>([&](auto J) {
        constexpr int j = decltype(J)::value;
        issue(s0 + j, std::integral_constant<int, j>{});
    });
    wait_vmcnt<(NST - 1) * DPS>();
    wg_barrier();
    read(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    for (int op = o_begin; op < o_end; op += TD) {
        static_for<0, TS>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int b = j % NST, r = j & 1, ch = j % NCH;
            constexpr bool odd = (j / NCH) & 1;
            const int s = op * NCH + j;
            // this wave's copies of step s + 1 are done, and every wave has
            // finished reading step s into registers
            wait_vmcnt<(NST - 2) * DPS>();
            wait_lgkm0();
            wg_barrier();
            __builtin_amdgcn_sched_barrier(0);
            // step s + 1 into the other register set (its latency runs under
            // this step's products)
            read(std::integral_constant<int, (j + 1) % NST>{}, std::integral_constant<int, 1 - r>{});
            const Copy cp = setup(s + NST, std::integral_constant<int, b>{});
            ACC &x0 = odd ? cb0 : ca0, &x1 = odd ? cb1 : ca1;
            if constexpr (ch == 0) x0 = x1 = ACC{};
            // products interleaved with the copies of step s + NST, in this
            // order (the matrix cores run while the copies are issued)
            static_for<0, NPR>([&](auto C) {
                constexpr int c = decltype(C)::value;
                product(std::integral_constant<int, r>{}, c, x0, x1);
                if constexpr (c < CH) copy_a(cp, c);
                __builtin_amdgcn_sched_barrier(0);
            });
            static_for<NPR, CH>([&](auto C) {
                copy_a(cp, decltype(C)::value);
            });
            static_for<0, BPW>([&](auto K) { copy_b(cp, decltype(K)::value); });
            if constexpr (ch == 0) {
                if constexpr (odd) run += ca0 + ca1;
                else run += cb0 + cb1;
            }
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    run += cb0 + cb1;   // the last displacement (TD is even)
    // no copy may still be writing LDS when the workgroup ends or reuses it
    wait_vmcnt<0>();
    wg_barrier();
    if constexpr (NSPLIT > 1) {
        ACC *red = reinterpret_cast<ACC *>(ring);   // [NSPLIT - 1][TPW][64]
        if (hs > 0) red[((hs - 1) * TPW + tw) * 64 + lane] = run;
        __syncthreads();
        if (hs > 0) return;
#pragma unroll
        for (int h = 0; h < NSPLIT - 1; ++h) run += red[(h * TPW + tw) * 64 + lane];
    }
    if (!active) return;

    // C[cell][node]: float, lane l, register r -> node j = l % 32, cell
    // ii = 4 (l / 32) + (r % 4) + 8 (r / 4); double, node j = l % 16, cell
    // ii = l / 16 + 4 r
    const int jn = nb * CELLS + (lane % CELLS);
    if (jn >= F::N3) return;
#pragma unroll
    for (int r = 0; r < F::REGS; ++r) {
        const int ii = F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 5) + (r & 3) + 8 * (r >> 2);
        const int64_t P2 = Pm0 + ii;
        if (P2 >= nparent) continue;
        const int x = 2 * compact3(P2) + px, y = 2 * compact3(P2 >> 1) + py, z = 2 * compact3(P2 >> 2) + pz;
        const int64_t c = x + int64_t(D) * (y + int64_t(D) * z);
        loc[c * NS + jn] = inv_side * run[r];
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

// LDS-staged far field: CH 16-byte pieces per lane and step, NST ring stages
template <int N, int MODE> struct MxLds {
    static constexpr int NA = MxForm<N, MODE>::NA;
    static constexpr int CH = NA % 4 == 0 ? 4 : 2;
    static constexpr int NST = 3;
};

// List split of a launch over levels [l0, l1] of tiles of `cells` parents:
// enough waves per tile to keep every SIMD busy.
int m2l_split_of(int n3, int cells, int l0, int l1)
{
    const int nb = (n3 + cells - 1) / cells;
    int64_t tiles = 0;
    for (int l = l0; l <= l1; ++l) {
        const int64_t Dp = (int64_t(1) << l) >> 1;
        tiles += 8 * nb * ((Dp * Dp * Dp + cells - 1) / cells);
    }
    return tiles >= 4096 ? 1 : (tiles >= 1024 ? 2 : 4);
}

}  // namespace

// Levels (bit l) whose interaction lists two workgroups share.  A launch
// with few tiles runs in a few rounds of equal workgroups, and the coarse
// levels' workgroups would form a last, mostly idle round; halved, they fill
// half a round.  Every level but the finest, in launches that split lists
// (not in the bf16 form).  The downward shifts add the two halves.
unsigned m2l_half_levels(const eqfmm_plan *plan)
{
    const Geom &g = plan->g;
    if (plan->p.precision == EQFMM_FP32_BF16FAR) return 0u;
    const int cells = plan->p.precision == EQFMM_FP64 ? 16 : 32;
    const int lmin = g.periodic ? 1 : 2;
    if (m2l_split_of(g.n3, cells, lmin, g.L) < 2) return 0u;
    unsigned m = 0;
    for (int l = lmin; l < g.L; ++l) m |= 1u << l;
    return m;
}

namespace {

// Level table of the LDS-staged kernel: one workgroup per (group of tpw
// tiles of `cells` parents, parity, node block[, list half]), levels finest
// first, each level's workgroups shared out evenly over the 8 XCDs.  Returns
// the grid size.
int fill_levels_tg(const Geom &g, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, int cells, int nb,
                   int tpw, unsigned halfmask, MxLevels &lv)
{
    lv.nlev = lmax - lmin + 1;
    int r = 0;
    for (int i = 0; i < lv.nlev; ++i) {
        const int l = lmax - i;
        const int Dp = (1 << l) >> 1;
        const int64_t nparent = int64_t(Dp) * Dp * Dp;
        lv.level[i] = l;
        lv.ntile[i] = int((nparent + cells - 1) / cells);
        lv.half[i] = int((halfmask >> l) & 1u);
        lv.nwg[i] = ((lv.ntile[i] + tpw - 1) / tpw * 8 * nb) << lv.half[i];
        lv.share[i] = (lv.nwg[i] + 7) / 8;
        lv.rbeg[i] = r;
        r += lv.share[i];
        lv.cell0[i] = lvl[l];
        lv.pcell0[i] = plvl[l];
        lv.inv_side[i] = float(double(1 << l) / g.box);
        lv.inv_side64[i] = double(1 << l) / g.box;
    }
    lv.rbeg[lv.nlev] = r;
    return 8 * r;
}

// The far-field products of levels [l0, l1] in one launch of form MODE.
template <int N, int MODE>
int launch_lds(eqfmm_plan *plan, int l0, int l1, const int64_t *lvl, const int64_t *plvl, const void *K,
               const void *phipad, void *loc, void *loc2, unsigned halfmask, hipStream_t st)
{
    using F = MxForm<N, MODE>;
    using C = MxLds<N, MODE>;
    const Geom &g = plan->g;
    if (halfmask && !loc2) return EQFMM_EINVAL;
    const int split = m2l_split_of(F::N3, F::CELLS, l0, l1);
    MxLevels lv;
    const int grid = fill_levels_tg(g, l0, l1, lvl, plvl, F::CELLS, F::NB, 4 / split, halfmask, lv);
    const int *tab = plan->ops.mxtab;
    if (split == 1)
        k_m2l_lds<N, MODE, C::CH, 1, C::NST><<<grid, 256, 0, st>>>(K, tab, lv, phipad, loc, loc2);
    else if (split == 2)
        k_m2l_lds<N, MODE, C::CH, 2, C::NST><<<grid, 256, 0, st>>>(K, tab, lv, phipad, loc, loc2);
    else
        k_m2l_lds<N, MODE, C::CH, 4, C::NST><<<grid, 256, 0, st>>>(K, tab, lv, phipad, loc, loc2);
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

template <int N>
int launch_mx(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const float *phipad,
              float *loc, float *loc2, hipStream_t st)
{
    const Geom &g = plan->g;
    // bf16 inputs only on the two finest levels, which carry nearly all the
    // work; on coarse levels the cells hold many charges and bf16 rounding of
    // their large, sign-cancelling vectors leaves a spurious net charge
    const bool bf = plan->p.precision == EQFMM_FP32_BF16FAR;
    const void *Kbf = static_cast<const unsigned char *>(plan->ops.Kmx) + mx_f32_bytes(g);
    if (!bf)
        return launch_lds<N, MX_F32>(plan, lmin, lmax, lvl, plvl, plan->ops.Kmx, phipad, loc, loc2,
                                     m2l_half_levels(plan), st);
    const int lb = lmax - 1 > lmin ? lmax - 1 : lmin;
    int rc = EQFMM_OK;
    if (lmin <= lb - 1)
        rc = launch_lds<N, MX_F32>(plan, lmin, lb - 1, lvl, plvl, plan->ops.Kmx, phipad, loc, loc2, 0u, st);
    return rc ? rc : launch_lds<N, MX_BF16>(plan, lb, lmax, lvl, plvl, Kbf, phipad, loc, loc2, 0u, st);
}

template <int N>
int launch_f64(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl,
               const double *phipad, double *loc, double *loc2, hipStream_t st)
{
    return launch_lds<N, MX_F64>(plan, lmin, lmax, lvl, plvl, plan->ops.Kmx, phipad, loc, loc2,
                                 m2l_half_levels(plan), st);
}

template <typename R, int N>
int launch_pad_n(const Geom &g, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const R *phi,
                 R *phipad, hipStream_t st)
{
    using V = typename std::conditional<sizeof(R) == sizeof(float), float4, double2>::type;
    constexpr int VPR = MxShape<N>::NS * int(sizeof(R)) / 16;
    MxPad pd;
    pd.nlev = lmax - lmin + 1;
    int64_t rows = 0;
    for (int i = 0; i < pd.nlev; ++i) {
        const int l = lmin + i;
        const int64_t P = (int64_t(1) << l) + 2 * kHalo;
        pd.level[i] = l;
        pd.row0[i] = rows;
        pd.src0[i] = lvl[l];
        pd.dst0[i] = plvl[l];
        rows += P * P * P;
    }
    pd.row0[pd.nlev] = rows;
    const int64_t blocks = (rows * VPR + 255) / 256;
    k_m2l_pad<V, VPR><<<dim3(unsigned(blocks)), 256, 0, st>>>(pd, g.periodic, reinterpret_cast<const V *>(phi),
                                                             reinterpret_cast<V *>(phipad));
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

}  // namespace

// The haloed copy of Phi at the interaction levels lmin..lmax.
template <typename R>
int launch_m2l_pad(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const R *phi,
                   R *phipad, hipStream_t st)
{
    const Geom &g = plan->g;
    if (lmax - lmin + 1 > 10 || lmin > lmax) return EQFMM_EINVAL;
    switch (g.n) {
        case 2: return launch_pad_n<R, 2>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        case 3: return launch_pad_n<R, 3>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        case 4: return launch_pad_n<R, 4>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        case 5: return launch_pad_n<R, 5>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        case 6: return launch_pad_n<R, 6>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        case 7: return launch_pad_n<R, 7>(g, lmin, lmax, lvl, plvl, phi, phipad, st);
        default: return EQFMM_EINVAL;
    }
}

// All interaction levels lmin..lmax in one launch (two for the bf16 mode);
// each writes (stores) its level's local vectors, the levels of
// m2l_half_levels as two halves, into loc and loc2.
template <typename R>
int launch_m2l(eqfmm_plan *plan, int lmin, int lmax, const int64_t *lvl, const int64_t *plvl, const R *phipad,
               R *loc, R *loc2, hipStream_t st)
{
    const Geom &g = plan->g;
    const int pk = prof_begin_m2l(plan, st);
    int rc = EQFMM_EINVAL;
#define EQ_CASE(NN)                                                                          \
    case NN:                                                                                 \
        if constexpr (sizeof(R) == sizeof(float))                                            \
            rc = launch_mx<NN>(plan, lmin, lmax, lvl, plvl, phipad, loc, loc2, st);          \
        else                                                                                 \
            rc = launch_f64<NN>(plan, lmin, lmax, lvl, plvl, phipad, loc, loc2, st);         \
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

template int launch_m2l_pad<float>(eqfmm_plan *, int, int, const int64_t *, const int64_t *, const float *, float *,
                                   hipStream_t);
template int launch_m2l_pad<double>(eqfmm_plan *, int, int, const int64_t *, const int64_t *, const double *,
                                    double *, hipStream_t);
template int launch_m2l<float>(eqfmm_plan *, int, int, const int64_t *, const int64_t *, const float *, float *,
                               float *, hipStream_t);
template int launch_m2l<double>(eqfmm_plan *, int, int, const int64_t *, const int64_t *, const double *,
                                double *, double *, hipStream_t);

}  // namespace eqfmm
