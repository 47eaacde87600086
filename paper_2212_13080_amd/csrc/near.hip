// Near field (a8) and far field at the charges (a7).  For every fragment:
// the direct sum over the same and the 26 adjacent finest cells (Sec. 1,
// Sec. 2.2 step 5), fragments of the same charge excluded; then Psi of its
// finest cell evaluated on the replacement of a unit charge there (Sec. 2.2
// step 4 and the force rule after step 5), added in a second kernel.  The
// direct sum needs only the binned charges, so it runs concurrently with the
// upward pass and the far field; the second kernel waits for the local
// vectors.
//
// Work decomposition of the direct sum: fragments are sorted by finest cell
// in row-major order (x fastest), so the cells x-1..x+1 of one row (y, z)
// are one contiguous range.  A workgroup owns RB consecutive cells of one
// x-row (about 64 targets).  When its 9 neighbouring rows hold at most
// kChunk sources, it stages them all in LDS at once and each target reads
// the sub-ranges of its own three cells per row, with S = 2 or 4 threads per
// target taking every S-th source (their sums are added in a fixed order at
// the end).  Dense blocks (clustered charges) read the same windows from
// global memory instead: the lanes of a wave then mostly share a cell and
// the loads are broadcasts.  Targets whose charge is split are evaluated in
// double even in the float modes (the force along a split axis is a short
// sum of large cancelling terms).  Near-field sums are kept in double until
// the far field is added.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace eqfmm {

namespace {

template <int N> struct NearShape {
    static constexpr int N3 = N * N * N;
    static constexpr int NS = (N3 + 15) & ~15;
};

// Compensated running sum (Knuth's two-sum): the rounding error of every
// addition is carried in c, so folding m block partials into it loses
// O(eps) in total instead of O(m eps).  Each per-target sum is two-level:
// plain sums over short blocks of sources (one neighbour segment, at most
// kBlock sources) or over one plane of basis nodes, folded in here.
template <typename C> struct CSum {
    C s = C(0), c = C(0);
    __device__ __forceinline__ void add(C x)
    {
        const C t = s + x;
        const C bp = t - s;
        c += (s - (t - bp)) + (x - bp);
        s = t;
    }
    __device__ __forceinline__ double value() const { return double(s) + double(c); }
};

constexpr int kBlock = 32;     // sources per plain block in the unstaged loops
constexpr int kChunk = 1024;   // staged sources of one row block
constexpr int kDense = 256;    // row blocks with this many targets go to k_near_dense
constexpr int kMaxRB = 64;     // cells per row block at most

template <int N, typename C, typename R>
__device__ __forceinline__ void l2p_part(const R *t_, const R *den_, const R *Lc, double ud, double vd,
                                         double wd, double inv_s, int sl, int S, double &ph, double &f0,
                                         double &f1, double &f2)
{
    C t[N], den[N], gx[N], gy[N], gz[N], dx[N], dy[N], dz[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        t[k] = C(t_[k]);
        den[k] = C(den_[k]);
    }
    const C u = C(ud), v = C(vd), w = C(wd);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        C p = C(1), dp = C(0), q = C(1), dq = C(0), r = C(1), dr = C(0);
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k != i) {
                dp = dp * (u - t[k]) + p;
                p = p * (u - t[k]);
                dq = dq * (v - t[k]) + q;
                q = q * (v - t[k]);
                dr = dr * (w - t[k]) + r;
                r = r * (w - t[k]);
            }
        gx[i] = den[i] * p;
        dx[i] = den[i] * dp;
        gy[i] = den[i] * q;
        dy[i] = den[i] * dq;
        gz[i] = den[i] * r;
        dz[i] = den[i] * dr;
    }
    CSum<C> a0, a1, a2, a3;
    for (int k = sl; k < N; k += S) {
        C b0 = C(0), b1 = C(0), b2 = C(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            C s0 = C(0), s1 = C(0);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const C l = C(Lc[i + N * j + N * N * k]);
                s0 += gx[i] * l;
                s1 += dx[i] * l;
            }
            b0 += gy[j] * s0;
            b1 += gy[j] * s1;
            b2 += dy[j] * s0;
        }
        a0.add(gz[k] * b0);
        a1.add(gz[k] * b1);
        a2.add(gz[k] * b2);
        a3.add(dz[k] * b0);
    }
    ph += a0.value();
    f0 -= a1.value() * inv_s;
    f1 -= a2.value() * inv_s;
    f2 -= a3.value() * inv_s;
}

template <typename R> __device__ __forceinline__ R rsqrt_t(R x);
// double: the hardware estimate refined by two Newton-Raphson steps for
// y = x^(-1/2) (y <- y + y (1 - x y^2) / 2, each step squaring the relative
// error), accurate to a few ulp for the positive normal r^2 of distinct charges
template <> __device__ __forceinline__ double rsqrt_t<double>(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
// the hardware reciprocal square root (1 ulp); r^2 of two distinct charges
// is never a float denormal at the box scales in use
template <> __device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// Coulomb term of one source at displacement (ex, ey, ez) = target - source;
// a fragment of the target's own charge (self included) adds exact zeros
template <typename C>
__device__ __forceinline__ void p2p_term(C ex, C ey, C ez, C q, bool self, C &ph, C &f0, C &f1, C &f2)
{
    const C r2 = self ? C(1) : ex * ex + ey * ey + ez * ez;
    const C ri = rsqrt_t<C>(r2);
    const C qr = (self ? C(0) : q) * ri;
    const C qr3 = qr * ri * ri;
    ph += qr;
    f0 += qr3 * ex;
    f1 += qr3 * ey;
    f2 += qr3 * ez;
}

// Staged sources [jl, jh), every S-th.  The displacement (target - source)
// is formed in double from cell-local coordinates: ex from xt - lx[j], where
// xt = target x + target cell and lx[j] = source x + its unwrapped cell (or,
// with UNWRAP false, from ud + (tx - ldx[j]) - lx[j] with lx the bare
// source x); self and same-charge pairs are recognised by the staged index
// oself (SELF_BY_INDEX, one fragment per charge) or by the owner.
template <typename C, typename R, bool UNWRAP, bool SELF_BY_INDEX>
__device__ __forceinline__ void p2p_range(const double *lx, const double *lv, const double *lw, const R *lq,
                                          const int *lpar, const int *ldx, int jl, int jh, int S, double xt,
                                          double ud, int tx, double vy, double wz, int par, int oself, double sd,
                                          C &ph, C &f0, C &f1, C &f2)
{
#pragma unroll 2
    for (int j = jl; j < jh; j += S) {
        const double dx = UNWRAP ? xt - lx[j] : ud + double(tx - ldx[j]) - lx[j];
        const C ex = C(dx * sd);
        const C ey = C((vy - lv[j]) * sd);
        const C ez = C((wz - lw[j]) * sd);
        const bool self = SELF_BY_INDEX ? j == oself : lpar[j] == par;
        p2p_term<C>(ex, ey, ez, C(lq[j]), self, ph, f0, f1, f2);
    }
}

// Sources [j0, j1) of one segment read from global memory (dense
// neighbourhoods), in plain blocks of kBlock folded into the compensated
// sums; targets evaluated in double (dbl) sum in double throughout.
template <typename R>
__device__ __forceinline__ void p2p_global(const double *su, const double *sv, const double *sw, const R *sq,
                                           const int *spar, const int *sleaf, int D, int j0, int j1, int shift,
                                           double ud, int tx, double vy, double wz, int par, bool dbl, double sd,
                                           CSum<R> &aph, CSum<R> &af0, CSum<R> &af1, CSum<R> &af2, double &dph,
                                           double &df0, double &df1, double &df2)
{
    for (int jb = j0; jb < j1; jb += kBlock) {
        const int je = jb + kBlock < j1 ? jb + kBlock : j1;
        R ph = R(0), f0 = R(0), f1 = R(0), f2 = R(0);
        for (int j = jb; j < je; ++j) {
            const double ex = ud + double(tx - ((sleaf[j] & (D - 1)) + shift)) - su[j];
            const double ey = vy - sv[j], ez = wz - sw[j];
            const bool self = spar[j] == par;
            if (dbl) p2p_term<double>(ex * sd, ey * sd, ez * sd, double(sq[j]), self, dph, df0, df1, df2);
            else p2p_term<R>(R(ex * sd), R(ey * sd), R(ez * sd), sq[j], self, ph, f0, f1, f2);
        }
        if (!dbl) {
            aph.add(ph);
            af0.add(f0);
            af1.add(f1);
            af2.add(f2);
        }
    }
}

// One segment of source cells in a neighbouring row: cells [lo, hi) of row
// base rb, whose unwrapped x index is the cell index + shift.
struct Seg {
    int rb, lo, hi, shift, dy, dz, r;
};

// the up to 27 segments (9 rows x main / left wrap / right wrap) of the
// row block [c0, c1) of row (y, z); returns their number
__device__ __forceinline__ int row_segments(const Geom &g, int y, int z, int c0, int c1, Seg *out)
{
    const int D = g.D;
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            int yy = y + dy, zz = z + dz;
            if (g.periodic) {
                yy = (yy + D) % D;
                zz = (zz + D) % D;
            } else if (yy < 0 || zz < 0 || yy >= D || zz >= D) {
                continue;
            }
            const int rb = (yy + D * zz) * D;
            const int r = 3 * (dz + 1) + (dy + 1);
            out[m++] = Seg{rb, c0 - 1 > 0 ? c0 - 1 : 0, c1 + 1 < D ? c1 + 1 : D, 0, dy, dz, r};
            if (g.periodic && c0 == 0) out[m++] = Seg{rb, D - 1, D, -D, dy, dz, r};
            if (g.periodic && c1 == D) out[m++] = Seg{rb, 0, 1, D, dy, dz, r};
        }
    return m;
}

// sources of target cell tx inside segment sg: [j0, j1)
__device__ __forceinline__ void window(const int *leafstart, const Seg &sg, int tx, int &j0, int &j1)
{
    int a = tx - 1 - sg.shift, b = tx + 1 - sg.shift;
    a = a > sg.lo ? a : sg.lo;
    b = b < sg.hi - 1 ? b : sg.hi - 1;
    if (a > b) {
        j0 = j1 = 0;
        return;
    }
    j0 = leafstart[sg.rb + a];
    j1 = leafstart[sg.rb + b + 1];
}

template <typename R>
__global__ void __launch_bounds__(256) k_near(Geom g, int RB, const int *leafstart, const double *su,
                                              const double *sv, const double *sw, const R *sq, const int *spar,
                                              const int *sleaf, const unsigned char *smask, double *sphi,
                                              double *snf)
{
    // float modes stage the unwrapped source x (cell + x) and so need no
    // per-source cell; double mode keeps the two apart (exact differences)
    constexpr bool UNWRAP = sizeof(R) == sizeof(float);
    __shared__ double lx[kChunk], lv[kChunk], lw[kChunk];
    __shared__ R lq[kChunk];
    __shared__ int lpar[kChunk], ldx[UNWRAP ? 1 : kChunk];
    __shared__ double red[3 * 4 * 64];   // slices 1..S-1, four sums, TT targets
    // the non-empty segments among 3r + kind of neighbour row r = 3 (dz + 1)
    // + (dy + 1): kind 0 is the cells c0-1 .. c1 of that row, kinds 1 and 2
    // the periodic images of cells D-1 and 0 beyond the walls
    __shared__ Seg segs[27];
    __shared__ int sbase[28], sj0[27], nseg_s;
    __shared__ int rls[9][kMaxRB + 3];   // leafstart of cells c0-1 .. c1+1 (clamped to [0, D]) of each row
    const int D = g.D;
    const int nxb = (D + RB - 1) / RB;
    const int row = blockIdx.x / nxb, xb = blockIdx.x - row * nxb;
    const int y = row % D, z = row / D;
    const int c0 = xb * RB, c1 = c0 + RB < D ? c0 + RB : D;
    const int T0 = leafstart[row * D + c0], T1 = leafstart[row * D + c1];
    const int T = T1 - T0;
    // empty blocks, and dense blocks (k_near_dense), leave at once (uniform)
    if (T == 0 || T >= kDense) return;
    const double sd = g.s_leaf;
    const bool mixed = sizeof(R) == sizeof(float) && g.continuous;
    auto row_base = [&](int r, bool &ok) {
        int yy = y + r % 3 - 1, zz = z + r / 3 - 1;
        if (g.periodic) {
            yy = (yy + D) % D;
            zz = (zz + D) % D;
            ok = true;
        } else {
            ok = yy >= 0 && zz >= 0 && yy < D && zz < D;
        }
        return (yy + D * zz) * D;
    };
    const int W = c1 - c0 + 3;
    for (int idx = threadIdx.x; idx < 9 * W; idx += 256) {
        const int r = idx / W, i = idx - r * W;
        bool ok;
        const int rb = row_base(r, ok);
        int c = c0 - 1 + i;
        c = c < 0 ? 0 : (c > D ? D : c);
        rls[r][i] = ok ? leafstart[rb + c] : 0;
    }
    if (threadIdx.x < 64) {   // wave 0: the non-empty segments, compacted, and their prefix
        const int k = threadIdx.x;
        int cnt = 0, j0 = 0;
        Seg sg{0, 0, 0, 0, 0, 0, 0};
        if (k < 27) {
            const int r = k / 3, kind = k - 3 * r;
            bool ok;
            const int rb = row_base(r, ok);
            sg = Seg{rb, 0, 0, 0, r % 3 - 1, r / 3 - 1, r};
            if (ok) {
                if (kind == 0) {
                    sg.lo = c0 - 1 > 0 ? c0 - 1 : 0;
                    sg.hi = c1 + 1 < D ? c1 + 1 : D;
                } else if (kind == 1 && g.periodic && c0 == 0) {
                    sg.lo = D - 1;
                    sg.hi = D;
                    sg.shift = -D;
                } else if (kind == 2 && g.periodic && c1 == D) {
                    sg.lo = 0;
                    sg.hi = 1;
                    sg.shift = D;
                }
            }
            if (sg.hi > sg.lo) {
                j0 = leafstart[rb + sg.lo];
                cnt = leafstart[rb + sg.hi] - j0;
            }
        }
        const bool live = sg.hi > sg.lo;
        const uint64_t mask = __ballot(live);
        const int pos = __popcll(mask & ((uint64_t(1) << k) - 1));
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (k >= off) incl += v;
        }
        if (live) {
            segs[pos] = sg;
            sj0[pos] = j0;
            sbase[pos] = incl - cnt;
        }
        if (k == 26) {
            nseg_s = __popcll(mask);
            sbase[__popcll(mask)] = incl;
        }
    }
    __syncthreads();
    const int nseg = nseg_s, nsrc = sbase[nseg];
    // Sparse blocks stage every source once in LDS and split each target over
    // S threads; dense neighbourhoods are read from global memory.
    const bool staged = nsrc <= kChunk;
    const int S = staged ? (T >= 128 ? 2 : 4) : 1;
    const int TT = 256 / S;
    const int tl = threadIdx.x % TT, sl = threadIdx.x / TT;
    if (staged) {
#pragma unroll
        for (int m = 0; m < kChunk / 256; ++m) {
            const int o = threadIdx.x + 256 * m;
            if (o >= nsrc) break;
            // the last segment that starts at or before o (it holds o)
            int k = 0;
#pragma unroll
            for (int step = 16; step > 0; step >>= 1)
                if (k + step < nseg && sbase[k + step] <= o) k += step;
            const int j = sj0[k] + (o - sbase[k]);
            const int dxc = (sleaf[j] & (D - 1)) + segs[k].shift;
            if constexpr (UNWRAP) {
                lx[o] = double(dxc) + su[j];
            } else {
                lx[o] = su[j];
                ldx[o] = dxc;
            }
            lv[o] = sv[j];
            lw[o] = sw[j];
            lq[o] = sq[j];
            lpar[o] = spar[j];
        }
        __syncthreads();
    }
    for (int tc = T0; tc < T1; tc += TT) {
        const int t = tc + tl;
        const bool act = t < T1;
        const int tt = act ? t : T0;
        const double ud = su[tt], vd = sv[tt], wd = sw[tt];
        const int par = spar[tt];
        const int leaf = sleaf[tt];
        const int tx = leaf & (D - 1);
        const double xt = ud + double(tx);
        const bool dbl = mixed && smask[par];
        CSum<R> aph, af0, af1, af2;
        double dph = 0.0, df0 = 0.0, df1 = 0.0, df2 = 0.0;
        if (act) {
            for (int k = 0; k < nseg; ++k) {
                const Seg sg = segs[k];
                // sources of cells tx-1 .. tx+1 in this segment, as global indices
                int j0, j1;
                if (sg.shift == 0) {
                    const int a = tx - 1 > sg.lo ? tx - 1 : sg.lo;
                    const int b = tx + 1 < sg.hi - 1 ? tx + 1 : sg.hi - 1;
                    if (a > b) continue;
                    j0 = rls[sg.r][a - (c0 - 1)];
                    j1 = rls[sg.r][b + 1 - (c0 - 1)];
                } else {
                    // an image cell beyond a wall neighbours only the cell at that wall
                    if (sg.shift < 0 ? tx != 0 : tx != D - 1) continue;
                    j0 = sj0[k];
                    j1 = j0 + (sbase[k + 1] - sbase[k]);
                }
                const double vy = vd - sg.dy, wz = wd - sg.dz;
                if (staged) {
                    R ph = R(0), f0 = R(0), f1 = R(0), f2 = R(0);
                    const int off = sbase[k] - sj0[k];
                    // one fragment per charge: the self pair is the target's own slot
                    const int oself = t + off;
                    if (dbl)
                        p2p_range<double, R, UNWRAP, false>(lx, lv, lw, lq, lpar, ldx, j0 + off + sl, j1 + off, S,
                                                            xt, ud, tx, vy, wz, par, oself, sd, dph, df0, df1, df2);
                    else if (g.continuous)
                        p2p_range<R, R, UNWRAP, false>(lx, lv, lw, lq, lpar, ldx, j0 + off + sl, j1 + off, S, xt,
                                                       ud, tx, vy, wz, par, oself, sd, ph, f0, f1, f2);
                    else
                        p2p_range<R, R, UNWRAP, true>(lx, lv, lw, lq, lpar, ldx, j0 + off + sl, j1 + off, S, xt,
                                                      ud, tx, vy, wz, par, oself, sd, ph, f0, f1, f2);
                    aph.add(ph);
                    af0.add(f0);
                    af1.add(f1);
                    af2.add(f2);
                } else {
                    p2p_global<R>(su, sv, sw, sq, spar, sleaf, D, j0, j1, sg.shift, ud, tx, vy, wz, par, dbl, sd,
                                  aph, af0, af1, af2, dph, df0, df1, df2);
                }
            }
        }
        // add the slices of each target in a fixed order
        double o0 = dbl ? dph : aph.value(), o1 = dbl ? df0 : af0.value();
        double o2 = dbl ? df1 : af1.value(), o3 = dbl ? df2 : af2.value();
        if (S > 1) {
            __syncthreads();
            if (sl > 0) {
                double *r = red + (sl - 1) * 4 * TT + tl;
                r[0] = o0;
                r[TT] = o1;
                r[2 * TT] = o2;
                r[3 * TT] = o3;
            }
            __syncthreads();
            if (sl == 0)
                for (int h = 0; h < S - 1; ++h) {
                    const double *r = red + h * 4 * TT + tl;
                    o0 += r[0];
                    o1 += r[TT];
                    o2 += r[2 * TT];
                    o3 += r[3 * TT];
                }
        }
        if (act && sl == 0) {
            sphi[t] = o0;
            snf[3 * int64_t(t) + 0] = o1;
            snf[3 * int64_t(t) + 1] = o2;
            snf[3 * int64_t(t) + 2] = o3;
        }
    }
}


// Targets of dense row blocks (>= kDense targets), one thread each over the
// sorted fragments: the lanes of a wave then mostly share a cell, so every
// source load is a broadcast, and a large cluster spreads over many waves.
template <typename R>
__global__ void __launch_bounds__(256) k_near_dense(Geom g, int RB, const int *nfrag, const int *leafstart,
                                                    const double *su, const double *sv, const double *sw,
                                                    const R *sq, const int *spar, const int *sleaf,
                                                    const unsigned char *smask, double *sphi, double *snf)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= *nfrag) return;
    const int D = g.D;
    const int leaf = sleaf[t];
    const int tx = leaf % D, row = leaf / D, y = row % D, z = row / D;
    const int c0 = (tx / RB) * RB, c1 = c0 + RB < D ? c0 + RB : D;
    if (leafstart[row * D + c1] - leafstart[row * D + c0] < kDense) return;
    const double sd = g.s_leaf;
    const double ud = su[t], vd = sv[t], wd = sw[t];
    const int par = spar[t];
    const bool dbl = sizeof(R) == sizeof(float) && g.continuous && smask[par];
    CSum<R> aph, af0, af1, af2;
    double dph = 0.0, df0 = 0.0, df1 = 0.0, df2 = 0.0;
    Seg segs[27];
    const int nseg = row_segments(g, y, z, tx, tx + 1, segs);
    for (int k = 0; k < nseg; ++k) {
        const Seg sg = segs[k];
        int j0, j1;
        window(leafstart, sg, tx, j0, j1);
        const double vy = vd - sg.dy, wz = wd - sg.dz;
        p2p_global<R>(su, sv, sw, sq, spar, sleaf, D, j0, j1, sg.shift, ud, tx, vy, wz, par, dbl, sd, aph, af0,
                      af1, af2, dph, df0, df1, df2);
    }
    sphi[t] = dbl ? dph : aph.value();
    snf[3 * t + 0] = dbl ? df0 : af0.value();
    snf[3 * t + 1] = dbl ? df1 : af1.value();
    snf[3 * t + 2] = dbl ? df2 : af2.value();
}

// Far field at the fragments (a7), added to their near-field sums: Psi of
// the fragment's finest cell evaluated on the replacement of a unit charge
// there, and its gradient.
template <int N, typename R>
__global__ void __launch_bounds__(256) k_l2p(Geom g, const R *t_, const R *den_, const int *nfrag, const double *su,
                                             const double *sv, const double *sw, const int *spar,
                                             const int *sleaf, const unsigned char *smask, const R *locL,
                                             double *sphi, const double *snf, R *sfld)
{
    using O = NearShape<N>;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= *nfrag) return;
    const double sd = g.s_leaf;
    const double ud = su[t], vd = sv[t], wd = sw[t];
    const bool dbl = sizeof(R) == sizeof(float) && g.continuous && smask[spar[t]];
    const R *Lc = locL + int64_t(sleaf[t]) * O::NS;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (dbl) l2p_part<N, double>(t_, den_, Lc, ud, vd, wd, 1.0 / sd, 0, 1, a0, a1, a2, a3);
    else l2p_part<N, R>(t_, den_, Lc, ud, vd, wd, 1.0 / sd, 0, 1, a0, a1, a2, a3);
    sphi[t] += a0;
    sfld[3 * t + 0] = R(snf[3 * t + 0] + a1);
    sfld[3 * t + 1] = R(snf[3 * t + 1] + a2);
    sfld[3 * t + 2] = R(snf[3 * t + 2] + a3);
}

}  // namespace

// cells per workgroup row block: about 64 targets on average
// n: charges (sets the row-block size); fcap: fragment capacity (grid of
// the dense kernel, which reads the actual count from leafstart[D^3])
template <typename R>
int launch_p2p(const eqfmm_plan *plan, int64_t n, int64_t fcap, const int *leafstart, const double *su,
               const double *sv, const double *sw, const R *sq, const int *spar, const int *sleaf,
               const unsigned char *smask, double *sphi, double *snf, hipStream_t st)
{
    const Geom &g = plan->g;
    const int64_t nleaf = int64_t(g.D) * g.D * g.D;
    const double mean = double(n) / double(nleaf);
    int RB = int(64.0 / (mean > 1e-9 ? mean : 1e-9) + 0.5);
    RB = RB < 1 ? 1 : (RB > g.D ? g.D : RB);
    RB = RB > kMaxRB ? kMaxRB : RB;
    const int nxb = (g.D + RB - 1) / RB;
    const int64_t grid = int64_t(g.D) * g.D * nxb;
    k_near<R><<<dim3(unsigned(grid)), 256, 0, st>>>(g, RB, leafstart, su, sv, sw, sq, spar, sleaf, smask, sphi,
                                                    snf);
    if (fcap > 0)
        k_near_dense<R><<<dim3(unsigned((fcap + 255) / 256)), 256, 0, st>>>(g, RB, leafstart + nleaf, leafstart, su,
                                                                           sv, sw, sq, spar, sleaf, smask, sphi,
                                                                           snf);
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

template <int N, typename R>
int launch_l2p(const eqfmm_plan *plan, int64_t fcap, const int *leafstart, const R *t, const R *den,
               const double *su, const double *sv, const double *sw, const int *spar, const int *sleaf,
               const unsigned char *smask, const R *locL, double *sphi, const double *snf, R *sfld, hipStream_t st)
{
    const int64_t nleaf = int64_t(plan->g.D) * plan->g.D * plan->g.D;
    if (fcap > 0)
        k_l2p<N, R><<<dim3(unsigned((fcap + 255) / 256)), 256, 0, st>>>(plan->g, t, den, leafstart + nleaf, su, sv,
                                                                        sw, spar, sleaf, smask, locL, sphi, snf,
                                                                        sfld);
    return hipGetLastError() == hipSuccess ? EQFMM_OK : EQFMM_EHIP;
}

template int launch_p2p<float>(const eqfmm_plan *, int64_t, int64_t, const int *, const double *, const double *,
                               const double *, const float *, const int *, const int *, const unsigned char *,
                               double *, double *, hipStream_t);
template int launch_p2p<double>(const eqfmm_plan *, int64_t, int64_t, const int *, const double *, const double *,
                                const double *, const double *, const int *, const int *, const unsigned char *,
                                double *, double *, hipStream_t);
#define EQ_L2P_INST(NN, RR)                                                                                  \
    template int launch_l2p<NN, RR>(const eqfmm_plan *, int64_t, const int *, const RR *, const RR *,         \
                                    const double *, const double *, const double *, const int *,            \
                                    const int *, const unsigned char *, const RR *, double *,               \
                                    const double *, RR *, hipStream_t);
EQ_L2P_INST(2, float) EQ_L2P_INST(3, float) EQ_L2P_INST(4, float) EQ_L2P_INST(5, float)
EQ_L2P_INST(6, float) EQ_L2P_INST(7, float)
EQ_L2P_INST(2, double) EQ_L2P_INST(3, double) EQ_L2P_INST(4, double) EQ_L2P_INST(5, double)
EQ_L2P_INST(6, double) EQ_L2P_INST(7, double)
#undef EQ_L2P_INST

}  // namespace eqfmm
