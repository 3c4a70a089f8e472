// stbem: HIP kernels for gfx950 and the host runtime behind include/stbem.h.
//
// Assembly (VALU-bound): one workgroup = one 16 x 16 tile of one causal
// block (k, m), k >= m; the upper blocks are never launched, and for the
// symmetric operators only the tiles on and above the block diagonal.  The
// time data of every block (lags, series coefficients) are built once per
// context; the far-field tiles read them and their Gauss rule from global
// memory (uniform, scalar loads), the touching-element tiles stage theirs in
// LDS with the singular-rule tables.  Lanes either compute one entry each or
// share piece-pair moments in LDS across the entries of the tile (V_h and D_h
// assembled together share D_h's tiles), and the lanes of a row store
// consecutive doubles.
// GEMV (HBM-bound): pass 1 computes one partial vector per stored block
// (8 rows per wavefront for A x, a lane per column for A^T x), pass 2 adds the
// partials of a block row (or column) in a fixed order, so results are
// bitwise reproducible.  GMRES keeps the Krylov basis in HBM; the small
// Hessenberg least-squares problem is solved on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "stbem_m0.h"
#include "stbem_tables.h"
#include "../../include/stbem.h"

using namespace stbem;

// ============================================================== kernels
namespace {

constexpr int kTile = 16;
constexpr int kWG = 256;

__device__ __forceinline__ void block_of(long long b, int& k, int& m)
{
    // b = k (k + 1) / 2 + m, 0 <= m <= k
    double s = sqrt(8.0 * (double)b + 1.0);
    long long kk = (long long)((s - 1.0) * 0.5);
    while (kk * (kk + 1) / 2 > b) --kk;
    while ((kk + 1) * (kk + 2) / 2 <= b) ++kk;
    k = (int)kk;
    m = (int)(b - kk * (kk + 1) / 2);
}

// V_h, dV_h/dalpha and D_h blocks are symmetric in space (the kernel of a
// block (k, m) is symmetric in x and y), so only the tiles (ti, tj) with
// ti <= tj are launched and an off-diagonal tile also stores its transpose.
constexpr bool sym_op(int op) { return op == OP_V || op == OP_DV || op == OP_D; }

inline long long tiles_per_block(int t1, bool sym) { return sym ? (long long)t1 * (t1 + 1) / 2 : (long long)t1 * t1; }

// tile number -> (ti, tj): row-major over all tiles, or over the upper triangle
__device__ __forceinline__ void tile_of(int tile, int t1, bool sym, int& ti, int& tj)
{
    if (!sym) { ti = tile / t1; tj = tile % t1; return; }
    int r = 0, n = t1;
    while (tile >= n) { tile -= n; ++r; --n; }
    ti = r; tj = r + tile;
}

// Matrix storage written by the assembly kernels: FP64, or FP32 (hi only),
// or the FP32 pair hi = fl32(v), lo = fl32(v - hi) that keeps about 48 bits.
// Which one is uniform over a launch, so the branch costs nothing per lane.
struct OutBuf {
    double* f64;
    float* hi;
    float* lo;
    __device__ __forceinline__ void put(long long e, double v) const
    {
        if (f64) { f64[e] = v; return; }
        const float h = (float)v;
        hi[e] = h;
        if (lo) lo[e] = (float)(v - (double)h);
    }
};

// Store the tile value of lane (il, jl) (entry (I0+il, J0+jl) of the block at
// boff).  For a symmetric operator an off-diagonal tile also stores its
// transposed tile, and a diagonal tile stores the values of its upper half
// (il <= jl) in both halves, staged through LDS so that the stores are
// row-contiguous and the stored blocks are exactly symmetric.  Every lane of
// the workgroup must call it.
__device__ __forceinline__ void store_tile(double (*stage)[kTile + 1], bool sym, double v, bool live, long long boff,
                                          int ng, int I0, int J0, int il, int jl, const OutBuf& out)
{
    if (!sym) {
        if (live) out.put(boff + (long long)(I0 + il) * ng + J0 + jl, v);
        return;
    }
    stage[il][jl] = v;
    __syncthreads();
    if (I0 == J0) {
        if (live) out.put(boff + (long long)(I0 + il) * ng + J0 + jl, il <= jl ? v : stage[jl][il]);
        return;
    }
    if (live) out.put(boff + (long long)(I0 + il) * ng + J0 + jl, v);
    const int r = J0 + il, col = I0 + jl;
    if (r < ng && col < ng) out.put(boff + (long long)r * ng + col, stage[jl][il]);
}

// lanes whose value a symmetric tile takes from the mirror: the lower half
// of a diagonal tile
__device__ __forceinline__ bool mirrored(bool sym, int I0, int J0, int il, int jl) { return sym && I0 == J0 && il > jl; }

// time data of every causal block (k, m), by packed index, once per context:
// the far-field tiles read it from global memory (uniform, scalar loads)
// instead of having one lane of every workgroup build it
__global__ __launch_bounds__(kWG) void k_time_blocks(Geom g, long long nb, TimeBlock* __restrict__ out)
{
    const long long b = (long long)blockIdx.x * kWG + threadIdx.x;
    if (b >= nb) return;
    int k, m;
    block_of(b, k, m);
    time_block(g, k, m, out[b]);
}

// The series data of separated time blocks for FP32 arithmetic (D_h's
// far field in the FP32-storage mode): the same coefficients as the FP64
// table (see TimeBlock), computed in FP64, truncated where p^(2n+2) < 1e-8
// (by the bound at kSeriesTol, the tail stays below 1.7e-8 of the leading
// coefficient: under FP32 rounding, 6e-8, and the FP32 far field's Gauss
// rule, about 3e-7) and stored as float.  nterm = 0 for blocks that are not
// series blocks.
constexpr double kSeriesTol32 = 1e-8;
struct TimeBlock32 {
    int nterm;
    float inv_dc;
    float pad[2];
    float st[kMaxTerms][12];
};

// gam_j of the rescaled Laguerre recurrence (time_block): gam_0 = gam_1 = 1,
// gam_{j+1} = j/(j+1) gam_{j-1}, i.e. prod over i = j-1, j-3, ... >= 1 of i/(i+1)
__device__ double lag_gamma(int j)
{
    double g = 1.0;
    for (int i = (j % 2 == 0) ? 1 : 2; i < j; i += 2) g *= (double)i / (i + 1);
    return g;
}

__global__ __launch_bounds__(kWG) void k_time_blocks32(Geom g, long long nb, TimeBlock32* __restrict__ out)
{
    const long long b = (long long)blockIdx.x * kWG + threadIdx.x;
    if (b >= nb) return;
    int k, m;
    block_of(b, k, m);
    TimeBlock32& tb = out[b];
    tb.nterm = 0;
    if (k - m < 2) return;
    const double hk = g.t[k + 1] - g.t[k], hm = g.t[m + 1] - g.t[m];
    const double A = 0.5 * hk, B = 0.5 * hm;
    const double dc = 0.5 * (g.t[k] + g.t[k + 1]) - 0.5 * (g.t[m] + g.t[m + 1]);
    const double p = (A + B) / dc, q = (A - B) / dc;
    if (p > 0.62) return;
    tb.inv_dc = (float)(1.0 / dc);
    const double p2 = p * p, q2 = q * q;
    int n = 0;
    for (double pp = p2; n < kMaxTerms; ++n) {
        if (n > 0 && pp < kSeriesTol32) { ++n; break; }
        pp *= p2;
    }
    tb.nterm = n;
    // tail sums kc, hc over the kept terms, as in time_block
    double kc = 0.0, hc = 0.0;
    for (int e = n - 1; e >= 0; --e) {
        const double cn = 2.0 * dc * dc * (pow(p2, e + 1) - pow(q2, e + 1)) / ((2.0 * e + 1.0) * (2.0 * e + 2.0));
        const double kc1 = e + 1 < n ? kc : 0.0;
        hc += kc1;
        const double hc1 = e + 1 < n ? hc : 0.0;
        kc += cn;
        hc += kc;
        // the rescaled recurrence of time_block: L_m = gam_m P_m
        const double g0 = lag_gamma(2 * e), g1 = lag_gamma(2 * e + 1);
        float* st = tb.st[e];
        st[6] = (float)(kc * g0); st[7] = (float)(kc1 * g1); st[8] = (float)(hc * g0); st[9] = (float)(hc1 * g1);
        st[10] = (float)((2.0 * e + 1.0) * cn * g1);
        st[11] = (float)(cn * g0);
        for (int h = 0; h < 2; ++h) {
            const int j = 2 * e - 1 + h;
            const double r = j >= 1 ? lag_gamma(j) / lag_gamma(j + 1) / (j + 1.0) : 0.0;
            st[3 * h] = (float)((2.0 * j + 1.0) * r);
            st[3 * h + 1] = (float)r;
            st[3 * h + 2] = 0.0f;
        }
    }
}

template <int OP>
__global__ __launch_bounds__(kWG) void k_assemble(Geom g, const Tables* __restrict__ Tg, Orders O,
                                                  double lmax, const int* __restrict__ blist, int tiles_1d,
                                                  OutBuf out, const TimeBlock* __restrict__ tbs)
{
    constexpr bool SYM = sym_op(OP);
    __shared__ Tables T;
    __shared__ int qf;
    __shared__ double stage[kTile][kTile + 1];
    const int tid = threadIdx.x;
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = tid; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    const long long tiles = SYM ? (long long)tiles_1d * (tiles_1d + 1) / 2 : (long long)tiles_1d * tiles_1d;
    const long long b = blist[blockIdx.x / tiles];
    int ti, tj;
    tile_of((int)(blockIdx.x % tiles), tiles_1d, SYM, ti, tj);
    int k, m;
    block_of(b, k, m);
    const TimeBlock& tb = tbs[b];
    if (tid == 0) qf = q_block(OP, lmax, block_min_lag(g.t, k, m), g.alpha);
    __syncthreads();
    const int il = tid / kTile, jl = tid % kTile, I0 = ti * kTile, J0 = tj * kTile;
    const int i = I0 + il, j = J0 + jl;
    const bool live = i < g.ng && j < g.ng, own = live && !mirrored(SYM, I0, J0, il, jl);
    double v = 0.0;
    if ((OP == OP_V || OP == OP_DV) && tb.d <= 1) {
        // touching time elements: the rules differ widely in cost (singular
        // rules for coincident and vertex-sharing segments, Gauss orders by
        // distance class), so the tile's entries are handed to the lanes in
        // order of cost and each wave meets one kind of work.  Every entry is
        // still computed by one lane with the same arithmetic.
        __shared__ int cnt[kMaxGL + 4];
        __shared__ short work[kWG];
        if (tid < kMaxGL + 4) cnt[tid] = 0;
        __syncthreads();
        int key = kMaxGL + 3;                                   // nothing to compute: last
        if (own) {
            const Piece P = seg_piece(g, i), Q = seg_piece(g, j);
            const int rel = relation(P, Q);
            key = rel == 1 ? 0 : rel >= 2 ? 1 : 2 + kMaxGL - q_touch(O, tb, P, Q, sep_ratio(P, Q), q_inc(OP));
        }
        const int rank = atomicAdd(&cnt[key], 1);
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int e = 0; e < kMaxGL + 4; ++e) { const int c = cnt[e]; cnt[e] = acc; acc += c; }
        }
        __syncthreads();
        work[cnt[key] + rank] = (short)(own ? tid : -1);
        __syncthreads();
        const int e = work[tid];
        double w = 0.0;
        if (e >= 0) w = entry<OP>(T, O, g, tb, qf, I0 + e / kTile, J0 + e % kTile);
        if (e >= 0) stage[e / kTile][e % kTile] = w;
        __syncthreads();
        v = own ? stage[il][jl] : 0.0;
        __syncthreads();
    } else if (own) {
        v = entry<OP>(T, O, g, tb, qf, i, j);
    }
    store_tile(stage, SYM, v, live, block_slot(g, b, k, m) * g.ng * g.ng, g.ng, I0, J0, il, jl, out);
}

// V_h, K_h and their alpha-derivatives on separated time elements (series),
// Gauss order Q fixed at compile time so the Q x Q node pairs of a segment
// pair unroll into Q independent series recurrences per step
// (instruction-level parallelism).  With z = alpha r^2 / (4 dc) and the sums
// S0 = sum c_n L_2n(z), S1 = sum c_n L^(1)_2n(z), S2 = sum c_n L^(2)_2n(z):
//   V  integrand  e^{-z} S0 / (4 pi dc)
//   K  integrand  (x-y).n_y alpha / (8 pi dc^2) e^{-z} S1
// and, as d/dalpha = (z / alpha) d/dz with d/dz (e^{-z} L^(b)_n) = -e^{-z} L^(b+1)_n,
//   dV integrand  -(z / alpha) e^{-z} S1 / (4 pi dc)
//   dK integrand  (x-y).n_y / (8 pi dc^2) e^{-z} (S1 - z S2)
//               = (x-y).n_y / (8 pi dc^2) e^{-z} SD,  SD = sum (2n+1) c_n L_2n+1(z)
// (z L^(2)_n = (n+2) L^(1)_n - (n+1) L^(1)_n+1 and L^(1)_n+1 - L^(1)_n = L_n+1):
// the series of the time kernel E1 that D_h's normal part uses, without the
// subtraction.
template <int Q, int OP>
__device__ __forceinline__ void far_pair(const Tables& T, const TimeBlock& tb, double al,
                                         const double* P, const double* Qs, double nqx, double nqy,
                                         double& m0, double& m1)
{
    // P, Qs: ax ay ex ey len; V, dV: m0 = int int of the kernel; K, dK: the
    // two shape moments of the double-layer kernel
    constexpr bool VT = OP == OP_V || OP == OP_DV;
    m0 = 0.0; m1 = 0.0;
#pragma unroll 1
    for (int a = 0; a < Q; ++a) {
        const double sP = P[4] * T.gl_x[Q][a];
        const double xx = P[0] + sP * P[2], xy = P[1] + sP * P[3];
        double z[Q], l0[Q], l1[Q], acc[Q], dn[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double sQ = Qs[4] * T.gl_x[Q][c];
            const double dx = xx - (Qs[0] + sQ * Qs[2]), dy = xy - (Qs[1] + sQ * Qs[3]);
            z[c] = 0.25 * al * (dx * dx + dy * dy) * tb.inv_dc;
            dn[c] = dx * nqx + dy * nqy;
            l0[c] = 1.0; l1[c] = 1.0 - z[c];
            acc[c] = OP == OP_V ? tb.st[0][11] : OP == OP_DK ? tb.st[0][10] * l1[c] : tb.st[0][6] + tb.st[0][7] * l1[c];
        }
        for (int n = 1; n < tb.nterm; ++n) {
            const double* st = tb.st[n];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const double x2 = fma(fma(-st[1], z[c], st[0]), l1[c], -l0[c]);
                const double x3 = fma(fma(-st[4], z[c], st[3]), x2, -l1[c]);
                if (OP == OP_V) acc[c] = fma(st[11], x2, acc[c]);
                else if (OP == OP_DK) acc[c] = fma(st[10], x3, acc[c]);
                else acc[c] = fma(st[7], x3, fma(st[6], x2, acc[c]));
                l0[c] = x2; l1[c] = x3;
            }
        }
        const double wP = P[4] * T.gl_w[Q][a];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double e = exp_neg(z[c], T.ex2);
            const double wq = wP * Qs[4] * T.gl_w[Q][c];
            if (OP == OP_V) {
                m0 += wq * e * acc[c];
            } else if (OP == OP_DV) {
                m0 += wq * e * z[c] * acc[c];
            } else {
                const double v = wq * dn[c] * e * acc[c];
                m0 += v * (1.0 - T.gl_x[Q][c]);
                m1 += v * T.gl_x[Q][c];
            }
        }
    }
    if (OP == OP_V) m0 *= tb.inv_dc * kInv4Pi;
    else if (OP == OP_DV) m0 *= -tb.inv_dc * kInv4Pi / al;
    else {
        const double f = (OP == OP_K ? al : 1.0) * 0.125 / kPi * tb.inv_dc * tb.inv_dc;
        m0 *= f; m1 *= f;
    }
}

template <int OP, int Q>
__global__ __launch_bounds__(kWG) void k_assemble_vkfar(Geom g, const Tables* __restrict__ Tg,
                                                        const int* __restrict__ blist, int tiles_i, int tiles_j,
                                                        OutBuf out, const TimeBlock* __restrict__ tbs)
{
    constexpr bool SYM = OP == OP_V || OP == OP_DV;
    constexpr bool KT = OP == OP_K || OP == OP_DK;     // hat columns (15 per tile)
    __shared__ double stage[kTile][kTile + 1];
    const int tid = threadIdx.x;
    const long long tiles = SYM ? (long long)tiles_i * (tiles_i + 1) / 2 : (long long)tiles_i * tiles_j;
    const long long b = blist[blockIdx.x / tiles];
    int ti, tj;
    if (SYM) tile_of((int)(blockIdx.x % tiles), tiles_i, true, ti, tj);
    else { const int tile = (int)(blockIdx.x % tiles); ti = tile / tiles_j; tj = tile % tiles_j; }
    int k, m;
    block_of(b, k, m);
    const TimeBlock& tb = tbs[b];
    const Tables& T = *Tg;                 // only the Q-point rule is read (uniform loads)
    const int ty = tid / kTile, tx = tid % kTile;
    const int i = ti * kTile + ty;
    // V: column j = J0 + tx.  K: the tile covers segments J0-1 .. J0+14 and
    // writes the 15 hats J0 .. J0+14 (hat j = rising part on j-1 + falling on j)
    const int J0 = tj * (KT ? kTile - 1 : kTile);
    int jseg = KT ? J0 - 1 + tx : J0 + tx;
    jseg = jseg < 0 ? jseg + g.ng : (jseg >= g.ng ? jseg - g.ng : jseg);
    double m0 = 0.0, m1 = 0.0;
    const bool live = i < g.ng && (KT || J0 + tx < g.ng);
    if (live && !mirrored(SYM, ti * kTile, J0, ty, tx)) {
        const double P[5] = {g.vx[i], g.vy[i], g.ex[i], g.ey[i], g.len[i]};
        const double Qs[5] = {g.vx[jseg], g.vy[jseg], g.ex[jseg], g.ey[jseg], g.len[jseg]};
        far_pair<Q, OP>(T, tb, g.alpha, P, Qs, g.ey[jseg], -g.ex[jseg], m0, m1);
    }
    const long long boff = block_slot(g, b, k, m) * g.ng * g.ng, rowoff = boff + (long long)i * g.ng;
    if (SYM) {
        store_tile(stage, true, m0, live, boff, g.ng, ti * kTile, J0, ty, tx, out);
    } else {
        // lanes of one tile row are consecutive: the rising moment of segment
        // j - 1 sits in the lane to the left
        const double left = __shfl_up(m1, 1, kTile);
        const int j = J0 + tx - 1;
        if (tx >= 1 && i < g.ng && j < g.ng) out.put(rowoff + j, left + m0);
    }
}

// K_h (and dK_h/dalpha) on touching time elements: like the far K tiles, a
// lane integrates one segment pair (row segment i, column segment J0-1+tx)
// once, with the rules for touching elements, for both trial shapes; hat j
// takes the rising moment of segment j-1 from the lane to its left.  Per hat
// this is one segment pair instead of two.
template <int OP>
__global__ __launch_bounds__(kWG, 3) void k_assemble_knear(Geom g, const Tables* __restrict__ Tg, Orders O,
                                                        const int* __restrict__ blist, int tiles_i, int tiles_j,
                                                        double* __restrict__ out64)
{
    __shared__ Tables T;
    __shared__ TimeBlock tb;
    const int tid = threadIdx.x;
    const long long tiles = (long long)tiles_i * tiles_j;
    const long long b = blist[blockIdx.x / tiles];
    const int tile = (int)(blockIdx.x % tiles);
    int k, m;
    block_of(b, k, m);
    if (tid == 0) time_block(g, k, m, tb);
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = tid; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    const int ty = tid / kTile, tx = tid % kTile;
    const int i = (tile / tiles_j) * kTile + ty;
    const int J0 = (tile % tiles_j) * (kTile - 1);
    int jseg = J0 - 1 + tx;
    jseg = jseg < 0 ? jseg + g.ng : (jseg >= g.ng ? jseg - g.ng : jseg);
    double m0 = 0.0, m1 = 0.0;
    if (i < g.ng) {
        const Piece P = seg_piece(g, i), Q = seg_piece(g, jseg);
        if (relation(P, Q) != 1) {          // coincident: (x-y).n = 0
            KernK<OP == OP_DK> kf(tb, g.alpha, Q);
            pair_integral(T, O, tb, 0, q_inc(OP), P, Q, kf);
            m0 = kf.acc0; m1 = kf.acc1;
        }
    }
    const double left = __shfl_up(m1, 1, kTile);
    const int j = J0 + tx - 1;
    if (tx >= 1 && i < g.ng && j < g.ng) out64[block_slot(g, b, k, m) * g.ng * g.ng + (long long)i * g.ng + j] = left + m0;
}

// D_h on separated time elements (series), one 16 x 16 tile of dual
// functions per workgroup.  The 2*16+2 half-segment pieces that carry the
// tile's rows (and columns) are paired once: each pair gets its four shape
// moments  int_P int_Q l_a(x) l_b(y) kappa(x, y),  l_0 = 1 - s/L, l_1 = s/L,
// with the raw hypersingular kernel kappa = alpha n_P.n_Q dF_D - t_P^T Hess(F_V) t_Q
// (smooth here); every entry then combines 4 x 4 pairs from LDS.
constexpr int kDP = 2 * kTile + 2;     // pieces per tile side

// four shape moments of the raw hypersingular kernel for one piece pair,
// Q x Q Gauss nodes, the Q series of a row of nodes advanced together
// WK: also the moments of K_h's kernel (x-y).n alpha e^{-z} S1 / (8 pi dc^2)
// (S1 = sum c_n L^(1)_2n, the sum the Hessian term already needs) in both
// orientations of the pair: kmom[0..1] = int int (x - y).n_Q G (1 - fy, fy)
// with fy the position of y along its whole segment (the piece is half hq of
// it), kmom[2..3] = int int (y - x).n_P G (1 - fx, fx) (half hp).  Unscaled:
// the caller multiplies by alpha / (8 pi dc^2).
template <int Q, bool WV, bool WK = false>
__device__ __forceinline__ void far_dpair(const Tables& T, const TimeBlock& tb, double al,
                                          const double* P, const double* Qs, double* mom, double* vmom,
                                          double* kmom = nullptr, int hp = 0, int hq = 0)
{
    const double cn = al * (P[5] * Qs[5] + P[6] * Qs[6]);
    const double tt = P[2] * Qs[2] + P[3] * Qs[3];
    // kappa = e^{-z} (fd sd + fk sk + fh zt s2), constants of the pair folded
    const double i1 = tb.inv_dc, i2 = i1 * i1, zf = 0.25 * al * i1;
    const double fd = -cn * i2 * kInv4Pi, fk = 0.5 * al * tt * i2 * kInv4Pi, fh = -0.25 * al * al * i2 * i1 * kInv4Pi;
    double m00 = 0, m01 = 0, m10 = 0, m11 = 0, mv = 0;
    double ka0 = 0, ka1 = 0, kb0 = 0, kb1 = 0;
#pragma unroll 1
    for (int a = 0; a < Q; ++a) {
        const double xa = T.gl_x[Q][a];
        const double sP = P[4] * xa, wP = P[4] * T.gl_w[Q][a];
        const double xx = P[0] + sP * P[2], xy = P[1] + sP * P[3];
        double z[Q], l0[Q], l1[Q], sd[Q], sk[Q], s2[Q], zt[Q], sv[Q], dna[Q], dnb[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double sQ = Qs[4] * T.gl_x[Q][c];
            const double dx = xx - (Qs[0] + sQ * Qs[2]), dy = xy - (Qs[1] + sQ * Qs[3]);
            z[c] = zf * (dx * dx + dy * dy);
            zt[c] = fh * ((dx * P[2] + dy * P[3]) * (dx * Qs[2] + dy * Qs[3]));
            if (WK) { dna[c] = dx * Qs[5] + dy * Qs[6]; dnb[c] = -(dx * P[5] + dy * P[6]); }
            l0[c] = 1.0; l1[c] = 1.0 - z[c];
            const double* s0 = tb.st[0];
            sd[c] = s0[10] * l1[c]; sk[c] = s0[6] + s0[7] * l1[c]; s2[c] = s0[8] + s0[9] * l1[c];
            if (WV) sv[c] = s0[11];
        }
        for (int n = 1; n < tb.nterm; ++n) {
            const double* st = tb.st[n];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const double x2 = fma(fma(-st[1], z[c], st[0]), l1[c], -l0[c]);
                const double x3 = fma(fma(-st[4], z[c], st[3]), x2, -l1[c]);
                sk[c] = fma(st[7], x3, fma(st[6], x2, sk[c]));
                s2[c] = fma(st[9], x3, fma(st[8], x2, s2[c]));
                sd[c] = fma(st[10], x3, sd[c]);
                if (WV) sv[c] = fma(st[11], x2, sv[c]);
                l0[c] = x2; l1[c] = x3;
            }
        }
        double r0 = 0, r1s = 0, rv = 0, ra0 = 0, ra1 = 0, rb = 0;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double e = exp_neg(z[c], T.ex2);
            const double kap = e * fma(zt[c], s2[c], fma(fk, sk[c], fd * sd[c]));
            const double xc = T.gl_x[Q][c], wq = Qs[4] * T.gl_w[Q][c];
            const double w = wq * kap;
            r0 = fma(w, 1.0 - xc, r0);
            r1s = fma(w, xc, r1s);
            if (WV) rv = fma(wq * e, sv[c], rv);
            if (WK) {
                const double gk = wq * e * sk[c], fy = 0.5 * (hq + xc);
                ra0 = fma(gk * dna[c], 1.0 - fy, ra0);
                ra1 = fma(gk * dna[c], fy, ra1);
                rb = fma(gk, dnb[c], rb);
            }
        }
        m00 += wP * (1.0 - xa) * r0; m01 += wP * (1.0 - xa) * r1s;
        m10 += wP * xa * r0;         m11 += wP * xa * r1s;
        if (WV) mv = fma(wP, rv, mv);
        if (WK) {
            const double fx = 0.5 * (hp + xa);
            ka0 = fma(wP, ra0, ka0); ka1 = fma(wP, ra1, ka1);
            kb0 = fma(wP * (1.0 - fx), rb, kb0); kb1 = fma(wP * fx, rb, kb1);
        }
    }
    mom[0] = m00; mom[1] = m01; mom[2] = m10; mom[3] = m11;
    if (WV) *vmom = mv * i1 * kInv4Pi;       // int int Delta F_V over the piece pair
    if (WK) { kmom[0] = ka0; kmom[1] = ka1; kmom[2] = kb0; kmom[3] = kb1; }
}

// K_h's kernel alone on one half-piece pair (the border pairs of the fused
// tile that only K_h needs): as far_dpair's kmom with the S1 series only;
// ORI = 0: int int (x - y).n_Q G fy, ORI = 1: int int (y - x).n_P G fx.
template <int Q, int ORI>
__device__ __forceinline__ double far_kpair(const Tables& T, const TimeBlock& tb, double al,
                                            const double* P, const double* Qs, int hp, int hq)
{
    const double zf = 0.25 * al * tb.inv_dc;
    double acc = 0.0;
#pragma unroll 1
    for (int a = 0; a < Q; ++a) {
        const double xa = T.gl_x[Q][a];
        const double sP = P[4] * xa, wP = P[4] * T.gl_w[Q][a];
        const double xx = P[0] + sP * P[2], xy = P[1] + sP * P[3];
        double z[Q], l0[Q], l1[Q], sk[Q], dn[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double sQ = Qs[4] * T.gl_x[Q][c];
            const double dx = xx - (Qs[0] + sQ * Qs[2]), dy = xy - (Qs[1] + sQ * Qs[3]);
            z[c] = zf * (dx * dx + dy * dy);
            dn[c] = ORI == 0 ? dx * Qs[5] + dy * Qs[6] : -(dx * P[5] + dy * P[6]);
            l0[c] = 1.0; l1[c] = 1.0 - z[c];
            sk[c] = tb.st[0][6] + tb.st[0][7] * l1[c];
        }
        for (int n = 1; n < tb.nterm; ++n) {
            const double* st = tb.st[n];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const double x2 = fma(fma(-st[1], z[c], st[0]), l1[c], -l0[c]);
                const double x3 = fma(fma(-st[4], z[c], st[3]), x2, -l1[c]);
                sk[c] = fma(st[7], x3, fma(st[6], x2, sk[c]));
                l0[c] = x2; l1[c] = x3;
            }
        }
        double r = 0.0;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const double xc = T.gl_x[Q][c], wq = Qs[4] * T.gl_w[Q][c];
            const double g = wq * exp_neg(z[c], T.ex2) * sk[c] * dn[c];
            r = fma(g, ORI == 0 ? 0.5 * (hq + xc) : 1.0, r);
        }
        acc = fma(ORI == 0 ? wP : wP * 0.5 * (hp + xa), r, acc);
    }
    return acc;
}


// WV: V_h on the same blocks from the same piece pairs (its kernel Delta F_V
// is one more series sum at the nodes D_h already evaluates): the 2 x 2 half
// pieces of segments I0 + s and J0 + r are pieces 2s+1, 2s+2 and 2r+1, 2r+2 of
// the tile, and V_h's tiles are the same symmetric 16 x 16 tiles.
// WK (with WV): K_h's separated blocks from the same node pairs too.  Its
// kernel needs only S1, which the Hessian term already sums, and the normal
// components of x - y.  A lane's segment pair (I0+il, J0+jl) gives, in both
// orientations, the falling and the rising moment of the trial hats on the
// trial segment; the hat of vertex n takes its rising part from segment n-1:
//   orientation A (K_h rows I0+il, hats J0+jl): from the lane on the left
//   (__shfl_up), for jl = 0 from the pairs of the pieces -1, 0 (the halves of
//   segment J0-1) computed by lanes 128..191;
//   orientation B (rows J0+jl, hats I0+il; off-diagonal tiles only, the
//   diagonal tile's A covers it): from the lane above through LDS, for il = 0
//   from the pieces -1, 0 of the row side (lanes 192..255).
// The piece arrays therefore start at piece -1.
template <int Q, bool WV, bool WK = false>
__global__ __launch_bounds__(kWG, (Q == 3 || (Q == 4 && !WV)) ? 3 : 1) void k_assemble_dfar(Geom g, const Tables* __restrict__ Tg,
                                                       const int* __restrict__ blist, int tiles_1d,
                                                       OutBuf out, OutBuf outv, const TimeBlock* __restrict__ tbs,
                                                       double* __restrict__ outk = nullptr)
{
    __shared__ double mom[kDP][kDP][4];
    __shared__ double pc[2][kDP + 1][7];   // pieces -1 .. kDP-1: ax ay ex ey len nx ny
    __shared__ double stage[kTile][kTile + 1];
    __shared__ double kb[WK ? 2 : 1][kTile][4];        // border K moments (A, B)
    __shared__ double kr[WK ? kTile : 1][kTile];        // orientation B rising moments
    const Tables& T = *Tg;                 // only the Q-point rule is read (uniform loads)
    const int tid = threadIdx.x;
    const long long tiles = (long long)tiles_1d * (tiles_1d + 1) / 2;
    const long long b = blist[blockIdx.x / tiles];
    int ti, tj;
    tile_of((int)(blockIdx.x % tiles), tiles_1d, true, ti, tj);
    int k, m;
    block_of(b, k, m);
    const TimeBlock& tb = tbs[b];
    const int I0 = ti * kTile, J0 = tj * kTile;
    const int np = 2 * g.ng;
    if (tid < 2 * (kDP + 1)) {
        int side = tid / (kDP + 1), u = tid % (kDP + 1) - 1;
        int base = side ? J0 : I0;
        int h = ((2 * base - 1 + u) % np + np) % np;
        Piece P = half_piece(g, h);
        double* q = pc[side][u + 1];
        q[0] = P.ax; q[1] = P.ay; q[2] = P.ex; q[3] = P.ey; q[4] = P.len; q[5] = P.nx; q[6] = P.ny;
    }
    __syncthreads();
    // lane (il, jl) takes the 2 x 2 pairs of pieces 2il+1, 2il+2 and 2jl+1,
    // 2jl+2 (the halves of segments I0+il and J0+jl, which give V_h's entry),
    // then lanes 0..131 one pair each on the border of the piece range
    const int il = tid / kTile, jl = tid % kTile, i = I0 + il, j = J0 + jl;
    double vsum = 0.0;
    double ka[2] = {0.0, 0.0}, kbo[2] = {0.0, 0.0};     // K moments of the lane's segment pair
#pragma unroll 1
    for (int e = 0; e < 4; ++e) {
        const int u = 2 * il + 1 + (e >> 1), v = 2 * jl + 1 + (e & 1);
        double vm = 0.0, km[4];
        far_dpair<Q, WV, WK>(T, tb, g.alpha, pc[0][u + 1], pc[1][v + 1], mom[u][v], &vm, km, e >> 1, e & 1);
        vsum += vm;
        if (WK) { ka[0] += km[0]; ka[1] += km[1]; kbo[0] += km[2]; kbo[1] += km[3]; }
    }
    if (tid < 4 * kDP - 4) {
        int u, v;
        if (tid < kDP) { u = 0; v = tid; }
        else if (tid < 2 * kDP) { u = kDP - 1; v = tid - kDP; }
        else if (tid < 3 * kDP - 2) { u = tid - 2 * kDP + 1; v = 0; }
        else { u = tid - (3 * kDP - 2) + 1; v = kDP - 1; }
        double unused;
        far_dpair<Q, false>(T, tb, g.alpha, pc[0][u + 1], pc[1][v + 1], mom[u][v], &unused);
    }
    if (WK && tid >= 128) {
        // border pairs of K_h: (pieces of row segment il) x (pieces -1, 0 of
        // column segment J0-1), or (pieces -1, 0 of row segment I0-1) x
        // (pieces of column segment jl)
        const int q = tid - 128, side = q >> 6, r = (q >> 2) & 15, sub = q & 3;
        if (side == 0)
            kb[0][r][sub] = far_kpair<Q, 0>(T, tb, g.alpha, pc[0][2 * r + 1 + (sub >> 1) + 1], pc[1][(sub & 1) - 1 + 1],
                                            sub >> 1, sub & 1);
        else if (I0 != J0)
            kb[1][r][sub] = far_kpair<Q, 1>(T, tb, g.alpha, pc[0][(sub >> 1) - 1 + 1], pc[1][2 * r + 1 + (sub & 1) + 1],
                                            sub >> 1, sub & 1);
    }
    if (WK) kr[il][jl] = kbo[1];
    __syncthreads();
    const bool live = i < g.ng && j < g.ng, own = live && !mirrored(true, I0, J0, il, jl);
    double acc = 0.0;
    if (own) {
        DualSupport si = dual_support(g, i), sj = dual_support(g, j);
        const int ui = 2 * il, vj = 2 * jl;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double a0 = si.v0[u], a1 = si.v0[u] + si.slope[u] * pc[0][ui + u + 1][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double b0 = sj.v0[v], b1 = sj.v0[v] + sj.slope[v] * pc[1][vj + v + 1][4];
                const double* M = mom[ui + u][vj + v];
                acc += a0 * (b0 * M[0] + b1 * M[1]) + a1 * (b0 * M[2] + b1 * M[3]);
            }
        }
    }
    const long long boff = block_slot(g, b, k, m) * g.ng * g.ng;
    store_tile(stage, true, acc, live, boff, g.ng, I0, J0, il, jl, out);
    if (WV) {
        __syncthreads();          // the stage is reused
        store_tile(stage, true, own ? vsum : 0.0, live, boff, g.ng, I0, J0, il, jl, outv);
    }
    if (WK) {
        const double f = g.alpha * 0.125 / kPi * tb.inv_dc * tb.inv_dc;
        // orientation A: row i, hat j = falling part on segment j + rising
        // part on segment j - 1
        const double left = __shfl_up(ka[1], 1, kTile);
        const double riseA = jl ? left : ((kb[0][il][0] + kb[0][il][1]) + kb[0][il][2]) + kb[0][il][3];
        if (live) outk[boff + (long long)i * g.ng + j] = f * (riseA + ka[0]);
        if (I0 != J0) {
            // orientation B: row j, hat i, through the stage (transposed store)
            const double riseB = il ? kr[il - 1][jl] : ((kb[1][jl][0] + kb[1][jl][1]) + kb[1][jl][2]) + kb[1][jl][3];
            __syncthreads();      // the stage is reused
            stage[jl][il] = f * (riseB + kbo[0]);
            __syncthreads();
            const int r = J0 + il, col = I0 + jl;
            if (r < g.ng && col < g.ng) outk[boff + (long long)r * g.ng + col] = stage[il][jl];
        }
    }
}

// D_h's far field in FP32 arithmetic (FP32-storage mode): the raw
// hypersingular kernel of far_dpair with the float series (TimeBlock32),
// node offsets formed from the pieces' start points in FP64 and rounded
// once, float moments and sums.  D_h only shapes the preconditioner.
constexpr float kInv4PiF = 0.0795774715459476679f;
template <int Q>
__device__ __forceinline__ void far_dpair32(const Tables& T, const TimeBlock32& tb, double al,
                                            const double* P, const double* Qs, float* mom)
{
    const float alf = (float)al;
    const float cn = (float)(al * (P[5] * Qs[5] + P[6] * Qs[6]));
    const float pex = (float)P[2], pey = (float)P[3], qex = (float)Qs[2], qey = (float)Qs[3];
    const float LP = (float)P[4], LQ = (float)Qs[4];
    const float tt = pex * qex + pey * qey;
    const float i1 = tb.inv_dc, i2 = i1 * i1, zf = 0.25f * alf * i1;
    const float fd = -cn * i2 * kInv4PiF, fk = 0.5f * alf * tt * i2 * kInv4PiF, fh = -0.25f * alf * alf * i2 * i1 * kInv4PiF;
    const float dx0 = (float)(P[0] - Qs[0]), dy0 = (float)(P[1] - Qs[1]);
    float m00 = 0.f, m01 = 0.f, m10 = 0.f, m11 = 0.f;
#pragma unroll 1
    for (int a = 0; a < Q; ++a) {
        const float xa = (float)T.gl_x[Q][a];
        const float sP = LP * xa, wP = LP * (float)T.gl_w[Q][a];
        const float bx = fmaf(sP, pex, dx0), by = fmaf(sP, pey, dy0);
        float z[Q], l0[Q], l1[Q], sd[Q], sk[Q], s2[Q], zt[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const float sQ = LQ * (float)T.gl_x[Q][c];
            const float dx = fmaf(-sQ, qex, bx), dy = fmaf(-sQ, qey, by);
            z[c] = zf * fmaf(dx, dx, dy * dy);
            zt[c] = fh * (fmaf(dx, pex, dy * pey) * fmaf(dx, qex, dy * qey));
            l0[c] = 1.f; l1[c] = 1.f - z[c];
            const float* s0 = tb.st[0];
            sd[c] = s0[10] * l1[c]; sk[c] = fmaf(s0[7], l1[c], s0[6]); s2[c] = fmaf(s0[9], l1[c], s0[8]);
        }
        for (int n = 1; n < tb.nterm; ++n) {
            const float* st = tb.st[n];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const float x2 = fmaf(fmaf(-st[1], z[c], st[0]), l1[c], -l0[c]);
                const float x3 = fmaf(fmaf(-st[4], z[c], st[3]), x2, -l1[c]);
                sk[c] = fmaf(st[7], x3, fmaf(st[6], x2, sk[c]));
                s2[c] = fmaf(st[9], x3, fmaf(st[8], x2, s2[c]));
                sd[c] = fmaf(st[10], x3, sd[c]);
                l0[c] = x2; l1[c] = x3;
            }
        }
        float r0 = 0.f, r1s = 0.f;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const float e = expf(-z[c]);
            const float kap = e * fmaf(zt[c], s2[c], fmaf(fk, sk[c], fd * sd[c]));
            const float xc = (float)T.gl_x[Q][c], w = LQ * (float)T.gl_w[Q][c] * kap;
            r0 = fmaf(w, 1.f - xc, r0);
            r1s = fmaf(w, xc, r1s);
        }
        m00 = fmaf(wP * (1.f - xa), r0, m00); m01 = fmaf(wP * (1.f - xa), r1s, m01);
        m10 = fmaf(wP * xa, r0, m10);         m11 = fmaf(wP * xa, r1s, m11);
    }
    mom[0] = m00; mom[1] = m01; mom[2] = m10; mom[3] = m11;
}

template <int Q>
__global__ __launch_bounds__(kWG) void k_assemble_dfar32(Geom g, const Tables* __restrict__ Tg,
                                                         const int* __restrict__ blist, int tiles_1d,
                                                         OutBuf out, const TimeBlock32* __restrict__ tbs)
{
    __shared__ float mom[kDP][kDP][4];
    __shared__ double pc[2][kDP][7];       // ax ay ex ey len nx ny
    __shared__ double stage[kTile][kTile + 1];
    const Tables& T = *Tg;
    const int tid = threadIdx.x;
    const long long tiles = (long long)tiles_1d * (tiles_1d + 1) / 2;
    const long long b = blist[blockIdx.x / tiles];
    int ti, tj;
    tile_of((int)(blockIdx.x % tiles), tiles_1d, true, ti, tj);
    int k, m;
    block_of(b, k, m);
    const TimeBlock32& tb = tbs[b];
    const int I0 = ti * kTile, J0 = tj * kTile;
    const int np = 2 * g.ng;
    if (tid < 2 * kDP) {
        int side = tid / kDP, u = tid % kDP;
        int base = side ? J0 : I0;
        int h = ((2 * base - 1 + u) % np + np) % np;
        Piece P = half_piece(g, h);
        double* q = pc[side][u];
        q[0] = P.ax; q[1] = P.ay; q[2] = P.ex; q[3] = P.ey; q[4] = P.len; q[5] = P.nx; q[6] = P.ny;
    }
    __syncthreads();
    // the same pair assignment as k_assemble_dfar: lane (il, jl) takes the
    // 2 x 2 pairs of pieces 2il+1, 2il+2 and 2jl+1, 2jl+2, then lanes
    // 0..131 one pair each on the border of the piece range
    const int il = tid / kTile, jl = tid % kTile, i = I0 + il, j = J0 + jl;
#pragma unroll 1
    for (int e = 0; e < 4; ++e) {
        const int u = 2 * il + 1 + (e >> 1), v = 2 * jl + 1 + (e & 1);
        far_dpair32<Q>(T, tb, g.alpha, pc[0][u], pc[1][v], mom[u][v]);
    }
    if (tid < 4 * kDP - 4) {
        int u, v;
        if (tid < kDP) { u = 0; v = tid; }
        else if (tid < 2 * kDP) { u = kDP - 1; v = tid - kDP; }
        else if (tid < 3 * kDP - 2) { u = tid - 2 * kDP + 1; v = 0; }
        else { u = tid - (3 * kDP - 2) + 1; v = kDP - 1; }
        far_dpair32<Q>(T, tb, g.alpha, pc[0][u], pc[1][v], mom[u][v]);
    }
    __syncthreads();
    const bool live = i < g.ng && j < g.ng, own = live && !mirrored(true, I0, J0, il, jl);
    float acc = 0.f;
    if (own) {
        DualSupport si = dual_support(g, i), sj = dual_support(g, j);
        const int ui = 2 * il, vj = 2 * jl;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float a0 = (float)si.v0[u], a1 = (float)(si.v0[u] + si.slope[u] * pc[0][ui + u][4]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float b0 = (float)sj.v0[v], b1 = (float)(sj.v0[v] + sj.slope[v] * pc[1][vj + v][4]);
                const float* M = mom[ui + u][vj + v];
                acc += a0 * fmaf(b0, M[0], b1 * M[1]) + a1 * fmaf(b0, M[2], b1 * M[3]);
            }
        }
    }
    store_tile(stage, true, (double)acc, live, block_slot(g, b, k, m) * g.ng * g.ng, g.ng, I0, J0, il, jl, out);
}

// D_h on touching time elements (d <= 1, closed form in time): one workgroup
// = one 16 x 16 tile.  Each of the 34 x 34 half-segment piece pairs of the
// tile enters up to four entries, so its moments are computed once into LDS.
// An entry takes the raw-kernel form when all 16 pairs of its supports are
// well separated, else the by-parts form (the boundary terms of the
// integration by parts cancel only within one entry, so the choice is per
// entry, never per pair).  The raw entries of the tile are done first, then,
// if the tile has any, the by-parts entries, reusing the moment array.
// WV: V_h's touching blocks from the same piece pairs (its kernel Delta F_V is
// the curl-term moment of the by-parts pairs and one more sum at the nodes of
// the raw pairs); V_h's entry (I0+s, J0+r) sums the pairs of pieces 2s+1,
// 2s+2 and 2r+1, 2r+2, which D_h's entry (s, r) needs as well.
template <bool WV>
__global__ __launch_bounds__(kWG) void k_assemble_dnear(Geom g, const Tables* __restrict__ Tg, Orders O,
                                                        const int* __restrict__ blist, int tiles_1d,
                                                        OutBuf out, OutBuf outv)
{
    __shared__ Tables T;
    __shared__ TimeBlock tb;
    __shared__ Piece pc[2][kDP];
    __shared__ double mom[kDP][kDP][5];
    __shared__ double vmom[WV ? kDP : 1][WV ? kDP : 1];   // int int Delta F_V per piece pair
    __shared__ unsigned char form[kTile][kTile];   // 0 by-parts, 1 raw, 2 outside the matrix
    __shared__ short list[kDP * kDP];              // pairs to compute, costly ones first
    __shared__ unsigned char keys[kDP * kDP];      // cost class of each pair
    __shared__ int cnt[kMaxGL + 3];
    __shared__ int nlist[2];
    __shared__ double stage[kTile][kTile + 1];
    const int tid = threadIdx.x;
    const long long tiles = (long long)tiles_1d * (tiles_1d + 1) / 2;
    const long long b = blist[blockIdx.x / tiles];
    int ti, tj;
    tile_of((int)(blockIdx.x % tiles), tiles_1d, true, ti, tj);
    int k, m;
    block_of(b, k, m);
    if (tid == 0) time_block(g, k, m, tb);
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = tid; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    const int I0 = ti * kTile, J0 = tj * kTile;
    const int np = 2 * g.ng;
    if (tid < 2 * kDP) {
        const int side = tid / kDP, u = tid % kDP;
        const int base = side ? J0 : I0;
        pc[side][u] = half_piece(g, ((2 * base - 1 + u) % np + np) % np);
    }
    __syncthreads();
    const int il = tid / kTile, jl = tid % kTile;
    const int i = I0 + il, j = J0 + jl;
    const bool inside = i < g.ng && j < g.ng;
    const int ui = 2 * il, vj = 2 * jl;
    int my = 2;
    if (inside) my = d_support_eta(&pc[0][ui], &pc[1][vj]) > O.eta_raw ? 1 : 0;
    form[il][jl] = (unsigned char)my;
    const int any_bp = __syncthreads_or(my == 0);

    // which form does a pair need: entries (u/2 - 1 or u/2, v/2 - 1 or v/2)
    auto needs = [&](int u, int v, int f) {
        const int i1 = u / 2, j1 = v / 2;
        bool r = false;
        for (int a = i1 - 1; a <= i1; ++a)
            for (int c = j1 - 1; c <= j1; ++c)
                if (a >= 0 && a < kTile && c >= 0 && c < kTile && form[a][c] == f) r = true;
        return r;
    };
    auto hat = [&](const DualSupport& sp, int u, double len, double& a0, double& a1) {
        a0 = sp.v0[u]; a1 = sp.v0[u] + sp.slope[u] * len;
    };
    DualSupport si, sj;
    if (inside) { si = dual_support(g, i); sj = dual_support(g, j); }
    double val = 0.0;

    // Pairs a pass needs, compacted so that no lane idles on unneeded pairs
    // and ordered by the cost of their rule (singular rules first, then by
    // Gauss order), so that the waves of one round meet one kind of work.
    // The order does not change any result: each pair's moments are
    // computed by one lane with the same arithmetic.
    auto build_list = [&](int f) {
        if (tid < kMaxGL + 3) cnt[tid] = 0;
        __syncthreads();
        for (int e = tid; e < kDP * kDP; e += kWG) {
            const int u = e / kDP, v = e % kDP;
            int key = kMaxGL + 2;                      // not needed by this pass
            if (needs(u, v, f)) {
                const Piece& P = pc[0][u];
                const Piece& Q = pc[1][v];
                key = relation(P, Q) ? 0 : 1 + kMaxGL - q_touch(O, tb, P, Q, sep_ratio(P, Q), 0);
                atomicAdd(&cnt[key], 1);
            }
            keys[e] = (unsigned char)key;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int c = 0; c < kMaxGL + 2; ++c) { const int n = cnt[c]; cnt[c] = acc; acc += n; }
            nlist[0] = acc;
        }
        __syncthreads();
        for (int e = tid; e < kDP * kDP; e += kWG) {
            const int key = keys[e];
            if (key < kMaxGL + 2) list[atomicAdd(&cnt[key], 1)] = (short)e;
        }
        __syncthreads();
        return nlist[0];
    };

    // pass 1: raw-form entries
    {
        const int n = build_list(1);
        for (int e = tid; e < n; e += kWG) {
            const int u = list[e] / kDP, v = list[e] % kDP;
            d_pair_raw<WV>(T, O, tb, g.alpha, pc[0][u], pc[1][v], mom[u][v], WV ? &vmom[WV ? u : 0][WV ? v : 0] : nullptr);
        }
    }
    __syncthreads();
    const bool mir = mirrored(true, I0, J0, il, jl);
    if (my == 1 && !mir) {
        double acc = 0.0;
        for (int u = 0; u < 4; ++u) {
            double a0, a1;
            hat(si, u, pc[0][ui + u].len, a0, a1);
            for (int v = 0; v < 4; ++v) {
                double b0, b1;
                hat(sj, v, pc[1][vj + v].len, b0, b1);
                const double* M = mom[ui + u][vj + v];
                acc += a0 * (b0 * M[0] + b1 * M[1]) + a1 * (b0 * M[2] + b1 * M[3]);
            }
        }
        val = acc;
    }
    if (any_bp) {
        __syncthreads();

        // pass 2: by-parts entries (curl part psi'_P psi'_Q m0 + the normal part)
        {
            const int n = build_list(0);
            for (int e = tid; e < n; e += kWG) {
                const int u = list[e] / kDP, v = list[e] % kDP;
                d_pair_bp(T, O, tb, g.alpha, pc[0][u], pc[1][v], mom[u][v]);
                if (WV) vmom[WV ? u : 0][WV ? v : 0] = mom[u][v][0];     // the curl-term moment is V's
            }
        }
        __syncthreads();
        if (my == 0 && !mir) {
            // the curl and the normal part of neighbouring dual functions
            // nearly cancel: every term goes into a compensated sum
            CSum acc = {0.0, 0.0};
            for (int u = 0; u < 4; ++u) {
                double a0, a1;
                hat(si, u, pc[0][ui + u].len, a0, a1);
                for (int v = 0; v < 4; ++v) {
                    double b0, b1;
                    hat(sj, v, pc[1][vj + v].len, b0, b1);
                    const double* M = mom[ui + u][vj + v];
                    acc.add(si.slope[u] * sj.slope[v] * M[0]);
                    acc.add(a0 * b0 * M[1]); acc.add(a0 * b1 * M[2]);
                    acc.add(a1 * b0 * M[3]); acc.add(a1 * b1 * M[4]);
                }
            }
            val = acc.value();
        }
    }
    const long long boff = block_slot(g, b, k, m) * g.ng * g.ng;
    store_tile(stage, true, val, inside, boff, g.ng, I0, J0, il, jl, out);
    if (WV) {
        double v = 0.0;
        if (inside && !mir) {
            const int u = 2 * il + 1, w = 2 * jl + 1;
            v = vmom[WV ? u : 0][WV ? w : 0] + vmom[WV ? u : 0][WV ? w + 1 : 0] +
                vmom[WV ? u + 1 : 0][WV ? w : 0] + vmom[WV ? u + 1 : 0][WV ? w + 1 : 0];
        }
        __syncthreads();          // the stage is reused
        store_tile(stage, true, v, inside, boff, g.ng, I0, J0, il, jl, outv);
    }
}

template <int OP>
__global__ __launch_bounds__(kWG) void k_entries(Geom g, const Tables* __restrict__ Tg, Orders O, double lmax,
                                                 long long n, const int* __restrict__ idx, double* __restrict__ out)
{
    __shared__ Tables T;
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= n) return;
    int k = idx[4 * e], m = idx[4 * e + 1], i = idx[4 * e + 2], j = idx[4 * e + 3];
    if (k < 0 || m < 0 || k >= g.nt || m >= g.nt || i < 0 || i >= g.ng || j < 0 || j >= g.ng) { out[e] = NAN; return; }   // outside the matrix
    if (k < m) { out[e] = 0.0; return; }
    TimeBlock tb;
    time_block(g, k, m, tb);
    int qf = q_block(OP, lmax, block_min_lag(g.t, k, m), g.alpha);
    out[e] = entry<OP>(T, O, g, tb, qf, i, j);
}

// M_h^0, pass 1: the three barycentric moments of every (row, triangle) pair
// of a chunk of rows into scratch[row - row0][t][v].
template <bool DERIV, bool FIRST, int PART = 0>
__global__ __launch_bounds__(kWG, PART == 2 ? 3 : 1) void k_m0_tri(Geom g, Mesh2 mesh, const Tables* __restrict__ Tg,
                                                const M0Tables* __restrict__ Dg, M0Orders MO, M0Poly PP,
                                                long long row0, long long lrow0, int nchunk,
                                                double* __restrict__ scratch)
{
    __shared__ Tables T;
    __shared__ M0Tables D;
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
        const double* s2 = reinterpret_cast<const double*>(Dg);
        double* d2 = reinterpret_cast<double*>(&D);
        for (int e = threadIdx.x; e < (int)(sizeof(M0Tables) / sizeof(double)); e += kWG) d2[e] = s2[e];
    }
    __syncthreads();
    const long long lrow = lrow0 + blockIdx.x / nchunk;       // row within the chunk
    int t = (int)(blockIdx.x % nchunk) * kWG + threadIdx.x;
    const long long row = row0 + lrow;          // row = k * ng + i
    const int k = (int)(row / g.ng), i = (int)(row % g.ng);
    if (FIRST || PP.n[k] > 0) {
        // The cost of a pair differs widely inside a row: in the first time
        // element the orders (up to 4^3 in nodes between near and far
        // triangles), in later ones the kernel (power series where
        // a = alpha r^2/4 <= amax, two E1 values beyond).  The workgroup's
        // triangles are handed to the lanes in order of cost, so that each
        // wave meets one kind of work (each triangle is still computed by one
        // lane with the same arithmetic).
        __shared__ int cnt[kMaxGL + 3];
        __shared__ int work[kWG];
        if (threadIdx.x < kMaxGL + 3) cnt[threadIdx.x] = 0;
        __syncthreads();
        int key = kMaxGL + 2;                                   // outside the mesh: last
        if (t < mesh.ntri) {
            const Piece S = seg_piece(g, i);
            const Tri3 tr = load_tri3(mesh, t);
            if (FIRST) {
                const int q0 = m0_first_order(MO, g, S, tr, 3);
                key = q0 == 0 ? 0 : 1 + kMaxGL - q0;            // near pairs, then by order
            } else {
                Tri tt;
                tt.ax = tr.ax; tt.ay = tr.ay; tt.bx = tr.bx; tt.by = tr.by; tt.cx = tr.cx; tt.cy = tr.cy;
                const double dlo = seg_tri_dist(S, tt);
                double dhi2 = 0.0;
                const double vx[3] = {tr.ax, tr.bx, tr.cx}, vy[3] = {tr.ay, tr.by, tr.cy};
                for (int e = 0; e < 2; ++e) {
                    const double px = S.ax + e * S.len * S.ex, py = S.ay + e * S.len * S.ey;
                    for (int v = 0; v < 3; ++v) dhi2 = fmax(dhi2, (vx[v] - px) * (vx[v] - px) + (vy[v] - py) * (vy[v] - py));
                }
                const double q4 = 0.25 * g.alpha, amax = PP.amax[k];
                key = q4 * dlo * dlo > amax ? 0 : (q4 * dhi2 <= amax ? 2 : 1);   // E1 only, mixed, series only
            }
        }
        const int rank = atomicAdd(&cnt[key], 1);
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int e = 0; e < kMaxGL + 3; ++e) { const int c = cnt[e]; cnt[e] = acc; acc += c; }
        }
        __syncthreads();
        work[cnt[key] + rank] = t;
        __syncthreads();
        t = work[threadIdx.x];
    }
    if (t >= mesh.ntri) return;
    if (FIRST && PART != 0) {
        // one kind of pair per launch: the other kind is left to the other launch
        const bool near = m0_first_order(MO, g, seg_piece(g, i), load_tri3(mesh, t), 3) == 0;
        if (near != (PART == 2)) return;
    }
    // k >= 1: the kernel varies on the time scale sqrt(4 t_k / alpha); k = 0:
    // the order follows the distance of the triangle (m0_tri_moments)
    int qs = 3;
    if (k > 0) {
        qs = q_time(fmax(g.len[i], MO.omax), g.t[k], g.alpha) + 1;
        qs = qs < 4 ? 4 : qs;
    }
    double mom[3];
    m0_tri_moments<DERIV, FIRST, PART>(T, D, MO, g, mesh, PP, k, i, t, qs, mom);
    double* o = scratch + (lrow * mesh.ntri + t) * 3;
    o[0] = mom[0]; o[1] = mom[1]; o[2] = mom[2];
}

// M0 rows of time elements k0 .. k0+nk-1 (k0 >= 1) for one segment and a
// chunk of triangles per workgroup: a lane takes one triangle for all these
// rows, in runs of rows with the same rule (at most kM0Group at a time), so
// that the E1 values at the shared time boundaries are computed once.
template <bool DERIV>
__global__ __launch_bounds__(kWG, 3) void k_m0_rows(Geom g, Mesh2 mesh, const Tables* __restrict__ Tg, M0Orders MO,
                                                 M0Poly PP, long long row0, int k0, int nk, int nchunk,
                                                 double* __restrict__ scratch)
{
    __shared__ Tables T;
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    const int i = (int)(blockIdx.x / nchunk);
    int t = (int)(blockIdx.x % nchunk) * kWG + threadIdx.x;
    {
        // the triangles are handed to the lanes in order of cost: the number
        // of rows that need E1 values (the others take the power series)
        constexpr int kKeys = 34;
        __shared__ int cnt[kKeys];
        __shared__ int work[kWG];
        if (threadIdx.x < kKeys) cnt[threadIdx.x] = 0;
        __syncthreads();
        int key = kKeys - 1;                                    // outside the mesh: last
        if (t < mesh.ntri) {
            const Piece S0 = seg_piece(g, i);
            const Tri3 t3 = load_tri3(mesh, t);
            double dhi2 = 0.0;
            const double vx[3] = {t3.ax, t3.bx, t3.cx}, vy[3] = {t3.ay, t3.by, t3.cy};
            for (int e = 0; e < 2; ++e) {
                const double px = S0.ax + e * S0.len * S0.ex, py = S0.ay + e * S0.len * S0.ey;
                for (int v = 0; v < 3; ++v) dhi2 = fmax(dhi2, (vx[v] - px) * (vx[v] - px) + (vy[v] - py) * (vy[v] - py));
            }
            const double ahi = 0.25 * g.alpha * dhi2;
            int ne = 0;
            for (int k = k0; k < k0 + nk; ++k) ne += (PP.n[k] == 0 || ahi > PP.amax[k]) ? 1 : 0;
            key = nk - ne;                                      // most E1 rows first
            key = key > kKeys - 2 ? kKeys - 2 : key;
        }
        const int rank = atomicAdd(&cnt[key], 1);
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int e = 0; e < kKeys; ++e) { const int c = cnt[e]; cnt[e] = acc; acc += c; }
        }
        __syncthreads();
        work[cnt[key] + rank] = t;
        __syncthreads();
        t = work[threadIdx.x];
    }
    if (t >= mesh.ntri) return;
    const Piece S = seg_piece(g, i);
    const Tri3 tr = load_tri3(mesh, t);
    auto order = [&](int k) {
        const int q = q_time(fmax(g.len[i], MO.omax), g.t[k], g.alpha) + 1;
        return q < 4 ? 4 : q;
    };
    for (int kk = k0; kk < k0 + nk;) {
        const int qs = order(kk);
        int run = 1;
        while (run < kM0Group && kk + run < k0 + nk && order(kk + run) == qs) ++run;
        double mom[3 * kM0Group];
        m0_rows_moments<DERIV>(T, g, PP, S, tr, kk, run, qs, mom);
#pragma unroll
        for (int r = 0; r < kM0Group; ++r) {
            if (r < run) {
                double* o = scratch + (((long long)(kk + r) * g.ng + i - row0) * mesh.ntri + t) * 3;
                o[0] = mom[3 * r]; o[1] = mom[3 * r + 1]; o[2] = mom[3 * r + 2];
            }
        }
        kk += run;
    }
}

// pass 2: M0[row][j] = sum over the triangles of vertex j (fixed order)
__global__ __launch_bounds__(kWG) void k_m0_gather(Mesh2 mesh, const int* __restrict__ v2t_loc, long long row0,
                                                   int nchunk, const double* __restrict__ scratch,
                                                   double* __restrict__ out)
{
    const long long lrow = blockIdx.x / nchunk;
    const int j = (int)(blockIdx.x % nchunk) * kWG + threadIdx.x;
    if (j >= mesh.nv) return;
    const double* sr = scratch + lrow * mesh.ntri * 3;
    double acc = 0.0;
    for (int p = mesh.v2t_ptr[j]; p < mesh.v2t_ptr[j + 1]; ++p) acc += sr[mesh.v2t[p] * 3 + v2t_loc[p]];
    out[(row0 + lrow) * mesh.nv + j] = acc;
}

// M_h^0 rows k >= ksplit: every (segment, triangle) pair lies in the range
// of the power series G_k = sc sum_n c_{k,n} a^n, a = alpha r^2/4, so the
// rows differ only by their coefficients.  The moments of a^n against the
// hats, S[i][n][t][v] = int_{gamma_i} int_t a^n lambda_v, are computed once
// with the quadrature the rows need at t_{ksplit} (the most demanding of
// them), gathered per vertex j into G[i][n][j], and every row is one
// contraction M0[(k,i), j] = sc sum_n c_{k,n} G[i][n][j].
// One lane per (segment, triangle, local vertex) of a chunk of segments.
__global__ __launch_bounds__(kWG) void k_m0_pow(Geom g, Mesh2 mesh, const Tables* __restrict__ Tg, double omax,
                                                double tsplit, int i0, int ni, int npow, double* __restrict__ S)
{
    __shared__ Tables T;
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    const long long per_i = 3LL * mesh.ntri;
    const long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= (long long)ni * per_i) return;
    const int il = (int)(e / per_i), rem = (int)(e % per_i), t = rem / 3, v = rem % 3;
    const int i = i0 + il;
    int qs = q_time(fmax(g.len[i], omax), tsplit, g.alpha) + 1;
    qs = qs < 4 ? 4 : qs;
    const Piece P = seg_piece(g, i);
    const Tri3 tr = load_tri3(mesh, t);
    const double e1x = tr.bx - tr.ax, e1y = tr.by - tr.ay, e2x = tr.cx - tr.ax, e2y = tr.cy - tr.ay;
    const double area2 = fabs(e1x * e2y - e1y * e2x), q4 = 0.25 * g.alpha;
    double mom[kPolyMax];
#pragma unroll
    for (int n = 0; n < kPolyMax; ++n) mom[n] = 0.0;
    for (int a = 0; a < qs; ++a) {
        const double u = T.gl_x[qs][a], wu = T.gl_w[qs][a] * (1.0 - u);
        for (int b = 0; b < qs; ++b) {
            const double vv = T.gl_x[qs][b] * (1.0 - u), w = wu * T.gl_w[qs][b] * area2;
            const double lam = v == 0 ? 1.0 - u - vv : (v == 1 ? u : vv);
            const double yx = tr.ax + u * e1x + vv * e2x, yy = tr.ay + u * e1y + vv * e2y;
            for (int c = 0; c < qs; ++c) {
                const double sx = P.len * T.gl_x[qs][c];
                const double dx = P.ax + sx * P.ex - yx, dy = P.ay + sx * P.ey - yy;
                const double aa = q4 * (dx * dx + dy * dy);
                double pw = w * lam * T.gl_w[qs][c];
#pragma unroll
                for (int n = 0; n < kPolyMax; ++n) {
                    if (n < npow) { mom[n] += pw; pw *= aa; }
                }
            }
        }
    }
#pragma unroll
    for (int n = 0; n < kPolyMax; ++n)
        if (n < npow) S[(((long long)il * npow + n) * mesh.ntri + t) * 3 + v] = mom[n] * P.len;
}

// G[i][n][j] = sum over the triangles of vertex j (fixed order)
__global__ __launch_bounds__(kWG) void k_m0_pow_gather(Mesh2 mesh, const int* __restrict__ v2t_loc, int i0, int ni,
                                                       int npow, const double* __restrict__ S, double* __restrict__ G)
{
    const long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= (long long)ni * npow * mesh.nv) return;
    const int j = (int)(e % mesh.nv);
    const long long ln = e / mesh.nv;          // il * npow + n
    const double* s = S + ln * mesh.ntri * 3;
    double acc = 0.0;
    for (int p = mesh.v2t_ptr[j]; p < mesh.v2t_ptr[j + 1]; ++p) acc += s[mesh.v2t[p] * 3 + v2t_loc[p]];
    G[((long long)i0 * npow + ln) * mesh.nv + j] = acc;
}

// rows k = ksplit .. nt-1: M0[(k,i), j] = sc sum_n coef[k][n] G[i][n][j]
__global__ __launch_bounds__(kWG) void k_m0_pow_apply(int ng, int nv, int nt, int ksplit, int npow,
                                                      const double* __restrict__ coef, double sc,
                                                      const double* __restrict__ G, double* __restrict__ out)
{
    const long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= (long long)ng * nv) return;
    const int i = (int)(e / nv), j = (int)(e % nv);
    double gm[kPolyMax];
#pragma unroll
    for (int n = 0; n < kPolyMax; ++n) gm[n] = n < npow ? G[((long long)i * npow + n) * nv + j] : 0.0;
    for (int k = ksplit; k < nt; ++k) {
        const double* ck = coef + (long long)k * kPolyMax;
        double acc = 0.0;
#pragma unroll
        for (int n = kPolyMax - 1; n >= 0; --n) acc += ck[n] * gm[n];
        out[((long long)k * ng + i) * nv + j] = sc * acc;
    }
}

// Representation formula (eq. (2)) at points (x, y, t): one workgroup per
// point.  Boundary potentials: the lanes take the (time element, segment)
// pairs with t_m < t in a fixed order; initial potential: the lanes take the
// triangles.  Sums are reduced in LDS in a fixed tree order.
__device__ __forceinline__ double block_reduce(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kWG / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kWG) void k_pot_bnd(Geom g, const Tables* __restrict__ Tg, Orders O,
                                                 const double* __restrict__ pts, const double* __restrict__ w,
                                                 const double* __restrict__ gd, int has_u0, double* __restrict__ out)
{
    __shared__ Tables T;
    __shared__ double red[kWG];
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    const long long p = blockIdx.x;
    const double x = pts[3 * p], y = pts[3 * p + 1], t = pts[3 * p + 2];
    int M = 0;
    while (M < g.nt && g.t[M] < t) ++M;
    double sl = 0.0, dl = 0.0;
    for (int e = threadIdx.x; e < M * g.ng; e += kWG) {
        const int m = e / g.ng, j = e % g.ng, jn = j + 1 == g.ng ? 0 : j + 1;
        const double shi = t - g.t[m], slo = fmax(t - g.t[m + 1], 0.0);
        const PotSeg r = pot_segment(T, O, g, j, x, y, slo, shi);
        const long long o = (long long)m * g.ng;
        sl += w[o + j] * r.sl;
        dl += gd[o + j] * r.d0 + gd[o + jn] * r.d1;
    }
    sl = block_reduce(sl, red);
    dl = block_reduce(dl, red);
    if (threadIdx.x == 0) {
        out[3 * p + 1] = sl;
        out[3 * p + 2] = dl;
        if (!has_u0) out[3 * p] = 0.0;
    }
}

__global__ __launch_bounds__(kWG) void k_pot_init(Geom g, Mesh2 mesh, const Tables* __restrict__ Tg, Orders O,
                                                  const double* __restrict__ pts, const double* __restrict__ u0,
                                                  double* __restrict__ out)
{
    __shared__ Tables T;
    __shared__ double red[kWG];
    {
        const double* src = reinterpret_cast<const double*>(Tg);
        double* dst = reinterpret_cast<double*>(&T);
        for (int e = threadIdx.x; e < (int)(sizeof(Tables) / sizeof(double)); e += kWG) dst[e] = src[e];
    }
    __syncthreads();
    const long long p = blockIdx.x;
    const double x = pts[3 * p], y = pts[3 * p + 1], t = pts[3 * p + 2];
    double acc = 0.0;
    for (int tri = threadIdx.x; tri < mesh.ntri; tri += kWG) {
        double mom[3];
        pot_triangle(T, O, g, mesh, tri, x, y, t, mom);
        for (int v = 0; v < 3; ++v) acc += u0[mesh.tri[3 * tri + v]] * mom[v];
    }
    acc = block_reduce(acc, red);
    if (threadIdx.x == 0) out[3 * p] = acc;
}

// ---------------------------------------------------------------- GEMV
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// vector loads of VW consecutive elements
template <class T, int VW>
struct VecLd {
    typedef T type __attribute__((ext_vector_type(VW)));
};

// partial[b][i] = sum_j A_b[i][j] x_m[j]: 4 waves x kRowsPerWave rows per
// workgroup, VW-wide loads (FP64 pair, hi+lo float pair, or FP32), ACC
// accumulation; the rows of a wave keep kRowsPerWave x CU loads per lane in
// flight (CU column chunks per step; each row still adds its chunks in
// column order).  The matrix is streamed once per product, so its loads are
// non-temporal.
constexpr int kRowsPerWave = 8;
template <class T, int VW, class ACC, bool HILO, int CU = 1>
__global__ __launch_bounds__(kWG) void k_gemv_n_vec(const T* __restrict__ A, const T* __restrict__ A2,
                                                    const double* __restrict__ x, double* __restrict__ part,
                                                    int ng, int rowchunks, long long b0)
{
    typedef typename VecLd<T, VW>::type VT;
    const long long b = b0 + blockIdx.x / rowchunks;
    const int rc = (int)(blockIdx.x % rowchunks);
    int k, m;
    block_of(b, k, m);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long base = b * (long long)ng * ng;
    const double* xm = x + (long long)m * ng;
    const int span = 64 * VW;
    const int i0 = (rc * 4 + wave) * kRowsPerWave;
    ACC s[kRowsPerWave];
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) s[rr] = 0;
    for (int c0 = lane * VW; c0 < ng; c0 += span * CU) {
        VT a[CU][kRowsPerWave], a2[HILO ? CU : 1][HILO ? kRowsPerWave : 1];
        ACC xv[CU][VW];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int c = c0 + u * span;
            if (c < ng) {
#pragma unroll
                for (int q = 0; q < VW; ++q) xv[u][q] = (ACC)xm[c + q];
#pragma unroll
                for (int rr = 0; rr < kRowsPerWave; ++rr) {
                    if (i0 + rr < ng) {
                        const long long o = base + (long long)(i0 + rr) * ng + c;
                        a[u][rr] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(A + o));
                        if (HILO) a2[HILO ? u : 0][HILO ? rr : 0] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(A2 + o));
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            if (c0 + u * span < ng) {
#pragma unroll
                for (int rr = 0; rr < kRowsPerWave; ++rr) {
                    if (i0 + rr < ng) {
                        if (HILO) {
#pragma unroll
                            for (int q = 0; q < VW; ++q) s[rr] += ((ACC)a[u][rr][q] + (ACC)a2[HILO ? u : 0][HILO ? rr : 0][q]) * xv[u][q];
                        } else {
#pragma unroll
                            for (int q = 0; q < VW; ++q) s[rr] += (ACC)a[u][rr][q] * xv[u][q];
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        ACC v = s[rr];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        const int i = i0 + rr;
        if (lane == 0 && i < ng) part[(b - b0) * ng + i] = (double)v;
    }
}

template <class T, int VW, class ACC, bool HILO>
__global__ __launch_bounds__(kWG) void k_gemv_t_vec(const T* __restrict__ A, const T* __restrict__ A2,
                                                    const double* __restrict__ x, double* __restrict__ part,
                                                    int ng, int colchunks, long long b0)
{
    typedef typename VecLd<T, VW>::type VT;
    __shared__ ACC red[4][64 * VW];
    const long long b = b0 + blockIdx.x / colchunks;
    const int cc = (int)(blockIdx.x % colchunks);
    int k, m;
    block_of(b, k, m);
    const int grp = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = cc * 64 * VW + lane * VW;
    const long long base = b * (long long)ng * ng;
    const double* xk = x + (long long)k * ng;
    ACC s[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) s[q] = 0;
    if (j0 < ng) {
#pragma unroll 4
        for (int i = grp; i < ng; i += 4) {
            const long long o = base + (long long)i * ng + j0;
            const ACC xi = (ACC)xk[i];
            VT a = __builtin_nontemporal_load(reinterpret_cast<const VT*>(A + o));
            if (HILO) {
                VT a2 = __builtin_nontemporal_load(reinterpret_cast<const VT*>(A2 + o));
#pragma unroll
                for (int q = 0; q < VW; ++q) s[q] += ((ACC)a[q] + (ACC)a2[q]) * xi;
            } else {
#pragma unroll
                for (int q = 0; q < VW; ++q) s[q] += (ACC)a[q] * xi;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < VW; ++q) red[grp][lane * VW + q] = s[q];
    __syncthreads();
    if (grp == 0 && j0 < ng) {
#pragma unroll
        for (int q = 0; q < VW; ++q) {
            const int c = lane * VW + q;
            part[(b - b0) * ng + j0 + q] = (double)(((red[0][c] + red[1][c]) + red[2][c]) + red[3][c]);
        }
    }
}

// y[k][i] = sum_{m<=k} part[b(k,m)][i]  (trans: y[m][j] = sum_{k>=m} part[b(k,m)][j])
// pass 2: y[(blk, i)] = sum of the partials of block row blk (column blk for
// the transpose).  A workgroup takes 32 outputs; 8 lanes per output sum
// fixed contiguous chunks of the partials, and the 8 chunk sums are added in
// chunk order, so the result does not depend on the launch.
// The partials present are those of the block rows [k0, k1), part[0] being
// packed block pb0 = k0 (k0 + 1) / 2.  trans = 0: outputs of block rows
// [k0, k1).  trans = 1: outputs of block columns [0, k1), summed over the
// rows k in [max(blk, k0), k1); a column's first rows (blk >= k0) write y,
// columns met in earlier row ranges (blk < k0) add to it.
constexpr int kRedSplit = 8, kRedOut = kWG / kRedSplit;
__global__ __launch_bounds__(kWG) void k_gemv_reduce(const double* __restrict__ part, double* __restrict__ y,
                                                     int ng, int k0, int k1, long long pb0, int trans)
{
    __shared__ double red[kRedSplit][kRedOut];
    const int seg = threadIdx.x / kRedOut, il = threadIdx.x % kRedOut;
    const long long e = (trans ? 0 : (long long)k0 * ng) + (long long)blockIdx.x * kRedOut + il;
    const long long eend = (long long)k1 * ng;
    double s = 0.0;
    int blk = 0;
    if (e < eend) {
        blk = (int)(e / ng);
        const int i = (int)(e % ng);
        const int lo = trans ? (blk > k0 ? blk : k0) : 0, len = trans ? k1 - lo : blk + 1;
        const int a = lo + (int)((long long)len * seg / kRedSplit), b = lo + (int)((long long)len * (seg + 1) / kRedSplit);
        if (!trans) {
            const long long b0 = (long long)blk * (blk + 1) / 2 - pb0;
            for (int m = a; m < b; ++m) s += part[(b0 + m) * ng + i];
        } else {
            for (int k = a; k < b; ++k) s += part[((long long)k * (k + 1) / 2 + blk - pb0) * ng + i];
        }
    }
    red[seg][il] = s;
    __syncthreads();
    if (seg == 0 && e < eend) {
        double t = red[0][il];
        for (int c = 1; c < kRedSplit; ++c) t += red[c][il];
        if (trans && blk < k0) y[e] += t;
        else y[e] = t;
    }
}

// Block-Toeplitz product (uniform time steps: block (k, m) = A_{k-m}, stored
// row-major at lag d = k - m).  With X, Y the N_Gamma x N_I views of x, y
// (column k = time element k):
//   TRANS = 0:  Y[i, k] = sum_{d <= k}        sum_j A_d[i, j] X[j, k - d]
//   TRANS = 1:  Y[j, m] = sum_{d < N_I - m}   sum_i A_d[i, j] X[i, m + d]
// a contraction over (d, j) (or (d, i)): it runs on the FP64 matrix cores.
// A workgroup owns a 64 x 64 tile of Y (rows x time columns), each of its
// four waves a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16
// (v_mfma_f64_16x16x4f64 on gfx950, layout measured: A operand lane =
// row + 16 kk, B operand lane = col + 16 kk, result register r of lane l =
// row l / 16 + 4 r, column l % 16).  The
// contraction index advances 16 at a time; lane kk of a 16-wide step takes
// the indices 4 kk .. 4 kk + 3, one per MFMA, so A's rows (TRANS = 0) and X's
// columns are read as 32-byte vectors when N_Gamma is a multiple of 16.
// The sum over (d, index) runs in one fixed order per output: results are
// bitwise reproducible.  Tiles are dealt to the 8 XCDs in runs that share
// a row strip of the A_d (L2 reuse), the longest lag ranges first.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTT = 64;            // tile edge
template <int TRANS, bool VEC>
__global__ __launch_bounds__(kWG) void k_toeplitz_mfma(const double* __restrict__ A, const double* __restrict__ x,
                                                       double* __restrict__ y, int ng, int nt, int tiles_r, int tiles_c)
{
    const int ntile = tiles_r * tiles_c;
    const int per = (ntile + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= ntile) return;
    const int rt = t / tiles_c, cslot = t % tiles_c;
    // TRANS = 0: column tiles with more lags (larger k) first; TRANS = 1: smaller m first
    const int ct = TRANS ? cslot : tiles_c - 1 - cslot;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = rt * kTT + (wave >> 1) * 32, c0 = ct * kTT + (wave & 1) * 32;
    const int lr = l & 15, kk = l >> 4;
    const long long ngl = ng, bsz = ngl * ngl;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    // lags that reach this wave's columns
    const int cmax = min(c0 + 31, nt - 1);
    if (c0 < nt && r0 < ng) {
        const int dend = TRANS ? nt - c0 : cmax + 1;
        for (int d = 0; d < dend; ++d) {
            const double* Ad = A + (long long)d * bsz;
            // time column of X feeding output column c: c - d (TRANS = 0) or c + d
            int xc[2];
            bool xok[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int c = c0 + b * 16 + lr;
                xc[b] = TRANS ? c + d : c - d;
                xok[b] = c < nt && xc[b] >= 0 && xc[b] < nt;
            }
            for (int j0 = 0; j0 < ng; j0 += 16) {
                const int jb = j0 + 4 * kk;          // this lane's 4 contraction indices
                double av[2][4], bv[2][4];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int row = r0 + a * 16 + lr;
                    if (!TRANS) {
                        // A_d[row][jb .. jb+3]
                        if (VEC && row < ng) {
                            const v4d q = *reinterpret_cast<const v4d*>(Ad + (long long)row * ng + jb);
                            av[a][0] = q[0]; av[a][1] = q[1]; av[a][2] = q[2]; av[a][3] = q[3];
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                av[a][q] = (row < ng && jb + q < ng) ? Ad[(long long)row * ng + jb + q] : 0.0;
                        }
                    } else {
                        // A_d[jb + q][row]: rows of A_d, 16 lanes read 16 consecutive columns
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            av[a][q] = (row < ng && jb + q < ng) ? Ad[(long long)(jb + q) * ng + row] : 0.0;
                    }
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double* xcol = x + (long long)xc[b] * ng;
                    if (VEC && xok[b]) {
                        const v4d q = *reinterpret_cast<const v4d*>(xcol + jb);
                        bv[b][0] = q[0]; bv[b][1] = q[1]; bv[b][2] = q[2]; bv[b][3] = q[3];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) bv[b][q] = (xok[b] && jb + q < ng) ? xcol[jb + q] : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][q], bv[b][q], acc[a][b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int c = c0 + b * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + a * 16 + kk + 4 * r;
                if (row < ng && c < nt) y[(long long)c * ng + row] = acc[a][b][r];
            }
        }
}

// dense row-major M (rows x cols): y = M x (a wavefront per row)
__global__ __launch_bounds__(kWG) void k_dense_n(const double* __restrict__ M, const double* __restrict__ x,
                                                 double* __restrict__ y, long long rows, int cols)
{
    const long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;
    double s = 0.0;
    for (int c = lane; c < cols; c += 64) s += M[r * cols + c] * x[c];
    s = wave_sum(s);
    if (lane == 0) y[r] = s;
}

// partials of y = M^T x over row chunks of 256
__global__ __launch_bounds__(kWG) void k_dense_t_part(const double* __restrict__ M, const double* __restrict__ x,
                                                      double* __restrict__ part, long long rows, int cols, int colchunks)
{
    const long long rc = blockIdx.x / colchunks;
    const int c = (int)(blockIdx.x % colchunks) * kWG + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    const long long r0 = rc * 256, r1 = r0 + 256 < rows ? r0 + 256 : rows;
    for (long long r = r0; r < r1; ++r) s += M[r * cols + c] * x[r];
    part[rc * cols + c] = s;
}

__global__ __launch_bounds__(kWG) void k_dense_t_reduce(const double* __restrict__ part, double* __restrict__ y,
                                                        int nrc, int cols)
{
    const int c = blockIdx.x * kWG + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int r = 0; r < nrc; ++r) s += part[(long long)r * cols + c];
    y[c] = s;
}

// ------------------------------------------------------- vector kernels
// (M g)[(k,i)] = h_k L_i / 2 (g[(k,i)] + g[(k,i+1)]);
// (M^T x)[(k,n)] = h_k / 2 (L_n x[(k,n)] + L_{n-1} x[(k,n-1)])
__global__ __launch_bounds__(kWG) void k_mass(const double* __restrict__ t, const double* __restrict__ len,
                                              const double* __restrict__ x, double* __restrict__ y, int ng, int nt,
                                              int trans, double scale, const double* __restrict__ addto)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= (long long)ng * nt) return;
    int k = (int)(e / ng), i = (int)(e % ng);
    double h = t[k + 1] - t[k];
    double v;
    if (!trans) {
        int ip = i + 1 == ng ? 0 : i + 1;
        v = 0.5 * h * len[i] * (x[(long long)k * ng + i] + x[(long long)k * ng + ip]);
    } else {
        int im = i == 0 ? ng - 1 : i - 1;
        v = 0.5 * h * (len[i] * x[(long long)k * ng + i] + len[im] * x[(long long)k * ng + im]);
    }
    y[e] = scale * v + (addto ? addto[e] : 0.0);
}

// y = a * x + b * y
__global__ __launch_bounds__(kWG) void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                                               double* __restrict__ y)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e < n) y[e] = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
}
__global__ __launch_bounds__(kWG) void k_fill(long long n, double v, double* __restrict__ y)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e < n) y[e] = v;
}

// y = x / d
__global__ __launch_bounds__(kWG) void k_div(long long n, const double* __restrict__ x, const double* __restrict__ d,
                                             double* __restrict__ y)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e < n) y[e] = x[e] / d[e];
}

// partial dot products: part[q * nchunk + c] = sum over chunk c of Q_q . v
constexpr int kDotChunk = 4096;
__global__ __launch_bounds__(kWG) void k_dots_part(const double* __restrict__ Q, long long ldq,
                                                   const double* __restrict__ v, long long n,
                                                   double* __restrict__ part, int nchunk)
{
    __shared__ double red[kWG / 64];
    const int c = blockIdx.x, q = blockIdx.y;
    const double* qq = Q + (long long)q * ldq;
    long long e0 = (long long)c * kDotChunk;
    long long e1 = e0 + kDotChunk < n ? e0 + kDotChunk : n;
    double s = 0.0;
    for (long long e = e0 + threadIdx.x; e < e1; e += kWG) s += qq[e] * v[e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)q * nchunk + c] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(kWG) void k_dots_reduce(const double* __restrict__ part, int nchunk, int nq,
                                                     double* __restrict__ out)
{
    int q = blockIdx.x * kWG + threadIdx.x;
    if (q >= nq) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)q * nchunk + c];
    out[q] = s;
}

// v -= sum_q Q_q h_q
__global__ __launch_bounds__(kWG) void k_basis_sub(const double* __restrict__ Q, long long ldq, int nq,
                                                   const double* __restrict__ h, double* __restrict__ v, long long n)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += Q[(long long)q * ldq + e] * h[q];
    v[e] -= s;
}

// w = sum_q Q_q y_q (+ w if accumulate)
__global__ __launch_bounds__(kWG) void k_basis_comb(const double* __restrict__ Q, long long ldq, int nq,
                                                    const double* __restrict__ y, double* __restrict__ w, long long n,
                                                    int accumulate)
{
    long long e = (long long)blockIdx.x * kWG + threadIdx.x;
    if (e >= n) return;
    double s = accumulate ? w[e] : 0.0;
    for (int q = 0; q < nq; ++q) s += Q[(long long)q * ldq + e] * y[q];
    w[e] = s;
}

// FP64 -> hi/lo FP32 split, FP64 -> FP32
__global__ __launch_bounds__(kWG) void k_split(long long n, const double* __restrict__ a, float* __restrict__ hi,
                                               float* __restrict__ lo)
{
    const long long stride = (long long)gridDim.x * kWG;
    for (long long e = (long long)blockIdx.x * kWG + threadIdx.x; e < n; e += stride) {
        double v = a[e];
        float h = (float)v;
        hi[e] = h;
        if (lo) lo[e] = (float)(v - (double)h);
    }
}

}  // namespace

// ============================================================ host side
// Device buffer of stbem_apply_noalloc: the partial vectors of a range of
// block rows.  One copy per GPU, held until the process ends; host code uses
// its address from hipGetSymbolAddress (per device), never the symbol itself.
constexpr long long kNoAllocDoubles = 1LL << 22;        // 32 MiB
static __device__ __align__(256) double noalloc_scratch[kNoAllocDoubles];
static_assert(kNoAllocDoubles * sizeof(double) == STBEM_NOALLOC_SCRATCH_BYTES, "scratch size and header disagree");

struct stbem_ctx {
    int ng = 0, nt = 0, nv = 0, ntri = 0;
    long long n = 0, nblk = 0, packed = 0;
    double alpha = 0, lmax = 0;
    std::vector<double> t, vx, vy, ex, ey, len, ox, oy;
    std::vector<int> tri, v2t_ptr, v2t, v2t_loc;
    // device copies
    double *d_t = nullptr, *d_vx = nullptr, *d_vy = nullptr, *d_ex = nullptr, *d_ey = nullptr, *d_len = nullptr;
    double *d_ox = nullptr, *d_oy = nullptr, *d_mt = nullptr;
    double *d_m0c = nullptr, *d_m0cd = nullptr, *d_m0amax = nullptr, *d_m0it = nullptr;
    double *d_m0ce = nullptr, *d_m0cde = nullptr, *d_m0es = nullptr;
    int m0_ksplit = 0, m0_npow = 0;   // M0 rows k >= m0_ksplit by moments of powers (none if == nt)
    int *d_m0n = nullptr, *d_v2t_loc = nullptr;
    int *d_tri = nullptr, *d_v2t_ptr = nullptr, *d_v2t = nullptr;
    Tables* d_tab = nullptr;
    TimeBlock* d_tbs = nullptr;         // the time data of every causal block, by packed index
    TimeBlock32* d_tbs32 = nullptr;     // float series data (FP32-storage mode), built on first use
    M0Tables* d_m0tab = nullptr;
    Orders ord;
    M0Orders m0ord;
    // operators
    double* mat[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};   // V K D M0 DV DK DM0
    size_t mat_bytes[7] = {0, 0, 0, 0, 0, 0, 0};
    // FP32 storage of V_h (hi, and lo when V_h has no FP64 storage) and D_h:
    // written by an assembly in STBEM_FP32_IR (then the FP64 storage of that
    // operator is not kept) or converted from FP64 storage (stbem_prepare_ir)
    float *v_hi = nullptr, *v_lo = nullptr, *d_32 = nullptr;
    // block lists per operator slot: [generic | far Q=3..8 (V, K) or tile kernel (D)]
    int* d_blist[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int nlist_touch[7] = {0, 0, 0, 0, 0, 0, 0};   // D_h: touching blocks for the tile kernel (list head)
    int nlist_gen[7] = {0, 0, 0, 0, 0, 0, 0};
    int nlist_far[7][9] = {};
    std::vector<int> list_nterm[7];       // series terms of each listed block (host copy, for the work model)
    std::vector<int> h_blist[7];          // host copy of the block lists (each group in increasing k)
    bool vd_fusable = false;              // V_h and D_h have the same far-tile block lists
    // K_h's blocks that are neither touching nor in D_h's far-tile lists: the
    // generic kernel takes them when K_h comes from D_h's far tiles
    int* d_klist_fused = nullptr;
    int nklist_fused = 0;
    // work
    double* part = nullptr;     // nblk * ng
    size_t part_bytes = 0;
    double* noalloc = nullptr;  // this device's noalloc_scratch (device address)
    double* wvec = nullptr;     // work vectors of N entries (right-hand side, preconditioner, solver)
    int wvec_count = 0;
    // GMRES workspace, kept between solves: Krylov basis (gm_cap + 1 vectors),
    // dot-product partials, Hessenberg column on the device, one vector
    double *gm_q = nullptr, *gm_part = nullptr, *gm_h = nullptr, *gm_v = nullptr;
    int gm_cap = 0;
    stbem_alloc_fn alloc = nullptr;
    stbem_free_fn release = nullptr;
    void* user = nullptr;
    std::string err;
    // block-Toeplitz storage (stbem_set_toeplitz): block (k, m) at lag k - m
    bool toep = false;
    // launch timing (stbem_set_timing): one event pair per launch
    struct TRec { std::string name; double units, flops; hipEvent_t a, b; };
    bool timing = false;
    std::vector<TRec> trecs;
};

namespace {

int fail(stbem_ctx* c, int code, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, expr)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail((c), STBEM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int op_slot(unsigned op)
{
    switch (op) {
    case STBEM_V: return 0;
    case STBEM_K: return 1;
    case STBEM_D: return 2;
    case STBEM_M0: return 3;
    case STBEM_DV: return 4;
    case STBEM_DK: return 5;
    case STBEM_DM0: return 6;
    }
    return -1;
}

void* dev_alloc(stbem_ctx* c, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (c->alloc) return c->alloc(bytes, c->user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    return p;
}

void dev_free(stbem_ctx* c, void* p)
{
    if (!p) return;
    if (c->release) c->release(p, c->user);
    else (void)hipFree(p);
}

template <class T>
int upload(stbem_ctx* c, T** dst, const std::vector<T>& src)
{
    size_t bytes = src.size() * sizeof(T);
    if (hipMalloc((void**)dst, bytes ? bytes : 8) != hipSuccess) return fail(c, STBEM_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    if (bytes) HIPCHK(c, hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice));
    return 0;
}

Geom geom(const stbem_ctx* c)
{
    Geom g;
    g.ng = c->ng; g.nt = c->nt; g.alpha = c->alpha;
    g.vx = c->d_vx; g.vy = c->d_vy; g.ex = c->d_ex; g.ey = c->d_ey; g.len = c->d_len; g.t = c->d_t;
    g.toep = c->toep ? 1 : 0;
    return g;
}

M0Poly m0poly(const stbem_ctx* c)
{
    M0Poly p;
    p.c = c->d_m0c; p.cd = c->d_m0cd; p.n = c->d_m0n; p.amax = c->d_m0amax; p.it = c->d_m0it;
    p.ce = c->d_m0ce; p.cde = c->d_m0cde; p.es = c->d_m0es;
    return p;
}

Mesh2 mesh(const stbem_ctx* c)
{
    Mesh2 m;
    m.nv = c->nv; m.ntri = c->ntri; m.ox = c->d_ox; m.oy = c->d_oy; m.tri = c->d_tri;
    m.v2t_ptr = c->d_v2t_ptr; m.v2t = c->d_v2t;
    return m;
}

inline long long grid1(long long n) { return (n + kWG - 1) / kWG; }

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int ensure_part(stbem_ctx* c)
{
    size_t need = (size_t)c->nblk * c->ng * sizeof(double);
    size_t need_dense = 0;
    if (c->nv > 0) need_dense = (size_t)((c->n + 255) / 256) * c->nv * sizeof(double);
    if (need_dense > need) need = need_dense;
    if (c->part && c->part_bytes >= need) return 0;
    if (c->part) (void)hipFree(c->part);
    c->part = nullptr;
    if (hipMalloc((void**)&c->part, need) != hipSuccess) { (void)hipGetLastError(); return fail(c, STBEM_ENOMEM, "work buffer of %zu bytes", need); }
    c->part_bytes = need;
    return 0;
}

// `count` work vectors of N doubles, kept by the context (allocated on first
// use, grown when a call needs more; the caller's stream order protects them:
// one context serves one stream)
int ensure_wvec(stbem_ctx* c, int count)
{
    if (c->wvec && c->wvec_count >= count) return 0;
    if (c->wvec) (void)hipFree(c->wvec);
    c->wvec = nullptr;
    c->wvec_count = 0;
    if (hipMalloc((void**)&c->wvec, (size_t)count * c->n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, STBEM_ENOMEM, "%d work vectors of %lld entries", count, c->n);
    }
    c->wvec_count = count;
    return 0;
}

// Brackets one kernel launch with HIP events on its stream when timing is on.
struct KTimer {
    stbem_ctx* c; hipStream_t s; long long idx = -1;
    KTimer(stbem_ctx* c_, const char* name, double units, hipStream_t s_, double flops = 0.0) : c(c_), s(s_)
    {
        if (!c->timing) return;
        stbem_ctx::TRec r{name, units, flops, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess) return;
        if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return; }
        (void)hipEventRecord(r.a, s);
        c->trecs.push_back(r);
        idx = (long long)c->trecs.size() - 1;
    }
    void stop()
    {
        if (idx >= 0) (void)hipEventRecord(c->trecs[idx].b, s);
        idx = -1;
    }
    ~KTimer() { stop(); }
};

void clear_timing(stbem_ctx* c)
{
    for (auto& r : c->trecs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    c->trecs.clear();
}

std::string kname(const char* base, int a) { return std::string(base) + "<" + std::to_string(a) + ">"; }
std::string kname(const char* base, int a, int b)
{
    return std::string(base) + "<" + std::to_string(a) + ", " + std::to_string(b) + ">";
}

// timer name of an assembly launch: the kernel's name, marked when the
// launch stores into FP32 storage (same kernel, 12 instead of 16 bytes per
// entry pair written)
std::string store_name(const char* base, const OutBuf& o)
{
    return o.f64 ? std::string(base) : std::string(base) + " f32-store";
}

// stored entries of a causal operator: packed lower block triangle, or one
// block per lag in block-Toeplitz mode
long long causal_entries(const stbem_ctx* c)
{
    return c->toep ? (long long)c->nt * c->ng * c->ng : c->packed;
}

// A dispatch's grid size is counted in work-items in 32 bits: launches over
// block lists are split so that workgroups x 256 stays below 2^32.
constexpr long long kMaxWG = (0xffffffffLL / kWG) - 1;

inline int blocks_per_launch(long long tiles)
{
    long long b = kMaxWG / (tiles > 0 ? tiles : 1);
    return (int)(b > 0x7fffffff ? 0x7fffffff : (b < 1 ? 1 : b));
}

// generic kernel over the block list from its touching part (with_touch,
// V_h assembled alone) or from its generic part
template <int OP>
int launch_assemble(stbem_ctx* c, OutBuf o64, hipStream_t s, bool with_touch = false)
{
    const int slot = OP == OP_V ? 0 : OP == OP_K ? 1 : OP == OP_D ? 2 : OP == OP_DV ? 4 : 5;
    int t1 = (c->ng + kTile - 1) / kTile;
    const long long tiles = tiles_per_block(t1, sym_op(OP));
    Geom g = geom(c);
    const int step = blocks_per_launch(tiles);
    const int first = with_touch ? 0 : c->nlist_touch[slot], count = c->nlist_gen[slot] + (with_touch ? c->nlist_touch[slot] : 0);
    for (int off = 0; off < count; off += step) {
        const int cnt = std::min(step, count - off);
        const int* bl = c->d_blist[slot] + first + off;
        dim3 gr((unsigned)(cnt * tiles)), blk(kWG);
        KTimer kt(c, kname("k_assemble", OP).c_str(), (double)cnt * g.ng * g.ng, s);
        hipLaunchKernelGGL((k_assemble<OP>), gr, blk, 0, s, g, c->d_tab, c->ord, c->lmax, bl, t1, o64, (const TimeBlock*)c->d_tbs);
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

// generic kernel over an explicit device list of blocks
template <int OP>
int launch_assemble_list(stbem_ctx* c, OutBuf o64, hipStream_t s, const int* list, int count)
{
    int t1 = (c->ng + kTile - 1) / kTile;
    const long long tiles = tiles_per_block(t1, sym_op(OP));
    Geom g = geom(c);
    const int step = blocks_per_launch(tiles);
    for (int off = 0; off < count; off += step) {
        const int cnt = std::min(step, count - off);
        dim3 gr((unsigned)(cnt * tiles)), blk(kWG);
        KTimer kt(c, kname("k_assemble", OP).c_str(), (double)cnt * g.ng * g.ng, s);
        hipLaunchKernelGGL((k_assemble<OP>), gr, blk, 0, s, g, c->d_tab, c->ord, c->lmax, list + off, t1, o64, (const TimeBlock*)c->d_tbs);
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

template <int OP>
void launch_knear(stbem_ctx* c, int slot, double* o, hipStream_t s)
{
    const int ti = (c->ng + kTile - 1) / kTile, tj = (c->ng + kTile - 2) / (kTile - 1);
    const long long tiles = (long long)ti * tj;
    const int step = blocks_per_launch(tiles);
    for (int off = 0; off < c->nlist_touch[slot]; off += step) {
        const int n = std::min(step, c->nlist_touch[slot] - off);
        KTimer kt(c, kname("k_assemble_knear", OP).c_str(), (double)n * c->ng * c->ng, s);
        hipLaunchKernelGGL((k_assemble_knear<OP>), dim3((unsigned)(n * tiles)), dim3(kWG), 0, s, geom(c), c->d_tab, c->ord,
                           (const int*)(c->d_blist[slot] + off), ti, tj, o);
    }
}

// Algorithmic operation counts of the far-field (series) kernels, FMA = 2,
// an FP64 exponential (exp_neg) = 19 (argument reduction 7, degree-5
// polynomial 10, table factor and scaling 2), counted from the kernels'
// arithmetic for the lanes that do work:
//   far_pair (V_h, K_h, dV_h, dK_h; one segment pair per lane): per row of
//     Q nodes 5; per node pair V 13 + 25 after the series, dV 14 + 28,
//     K 18 + 29, dK 17 + 29; per series term and node pair V and dK 10, K and
//     dV 12 (two rescaled recurrence steps of 4, sums 2 or 4)
//   far_dpair (D_h; one half-piece pair): 21 per pair; per row 19 (WV) or
//     17; per node pair 25 + 35 (WV) or 32 after the series; per term 20 (WV)
//     or 18; per stored D_h entry of a tile 196 to combine 16 pairs (+3 V_h)
// sum_nterm is the sum of the series terms of the launched blocks.
double flops_vkfar(int op, int Q, long long nblk, long long sum_nterm, long long lanes_per_block)
{
    const double q2 = (double)Q * Q;
    const double node = op == OP_V ? 38.0 : op == OP_DV ? 42.0 : op == OP_K ? 47.0 : 46.0;
    const double term = op == OP_V || op == OP_DK ? 10.0 : 12.0;
    return (double)lanes_per_block * ((double)nblk * (5.0 * Q + q2 * (node - term) + 5.0) + term * q2 * (double)sum_nterm);
}

double flops_dfar(int Q, bool wv, long long nblk, long long sum_nterm, long long tiles_per_blk, long long owned_per_blk,
                  bool wk = false)
{
    const double q2 = (double)Q * Q;
    const double pw = wv ? 1024.0 : 0.0, pp = wv ? 132.0 : 1156.0;       // pairs per tile with / without V_h
    double per_pair_wv = 21.0 + 19.0 * Q + q2 * (60.0 - 20.0), per_pair = 21.0 + 17.0 * Q + q2 * (57.0 - 18.0);
    const double tiles = (double)tiles_per_blk;
    double kborder = 0.0;
    if (wk) {
        // K_h moments: per node pair 20 (normal components 6, weight 2,
        // shape 2, four moments 10), per row 12; border pairs (64 per tile,
        // 128 off the diagonal): per node pair 20 + 12 per series term, per row 4
        per_pair_wv += 12.0 * Q + 20.0 * q2;
        const double border = 64.0 + 128.0 * (tiles - 1.0) / tiles;
        kborder = tiles * border * ((double)nblk * (4.0 * Q + 20.0 * q2) + 12.0 * q2 * (double)sum_nterm);
    }
    return tiles * (pw * ((double)nblk * per_pair_wv + 20.0 * q2 * (double)sum_nterm) +
                    pp * ((double)nblk * per_pair + 18.0 * q2 * (double)sum_nterm)) + kborder +
           (double)nblk * (double)owned_per_blk * (wv ? (wk ? 215.0 : 199.0) : 196.0);
}

long long sum_terms(const stbem_ctx* c, int slot, const int* bl, int cnt)
{
    const long long off = bl - c->d_blist[slot];
    long long sum = 0;
    for (int e = 0; e < cnt; ++e) sum += c->list_nterm[slot][off + e];
    return sum;
}

template <int OP, int Q>
void launch_vkfar(stbem_ctx* c, int slot, const int* bl, int cnt, OutBuf o, hipStream_t s)
{
    constexpr bool SYM = OP == OP_V || OP == OP_DV;
    int ti = (c->ng + kTile - 1) / kTile;
    int tj = SYM ? ti : (c->ng + kTile - 2) / (kTile - 1);
    const long long tiles = SYM ? tiles_per_block(ti, true) : (long long)ti * tj;
    const int step = blocks_per_launch(tiles);
    for (int off = 0; off < cnt; off += step) {
        const int n = std::min(step, cnt - off);
        const long long lanes = SYM ? (long long)c->ng * (c->ng + 1) / 2 : (long long)c->ng * tj * kTile;
        KTimer kt(c, kname("k_assemble_vkfar", OP, Q).c_str(), (double)n * c->ng * c->ng, s,
                  c->timing ? flops_vkfar(OP, Q, n, sum_terms(c, slot, bl + off, n), lanes) : 0.0);
        hipLaunchKernelGGL((k_assemble_vkfar<OP, Q>), dim3((unsigned)(n * tiles)), dim3(kWG), 0, s, geom(c), c->d_tab,
                           bl + off, ti, tj, o, (const TimeBlock*)c->d_tbs);
    }
}

template <int OP>
int launch_far(stbem_ctx* c, int slot, OutBuf o, hipStream_t s)
{
    const int* bl = c->d_blist[slot] + c->nlist_touch[slot] + c->nlist_gen[slot];
    int off = 0;
    launch_vkfar<OP, 3>(c, slot, bl + off, c->nlist_far[slot][3], o, s); off += c->nlist_far[slot][3];
    launch_vkfar<OP, 4>(c, slot, bl + off, c->nlist_far[slot][4], o, s); off += c->nlist_far[slot][4];
    launch_vkfar<OP, 5>(c, slot, bl + off, c->nlist_far[slot][5], o, s); off += c->nlist_far[slot][5];
    launch_vkfar<OP, 6>(c, slot, bl + off, c->nlist_far[slot][6], o, s); off += c->nlist_far[slot][6];
    launch_vkfar<OP, 7>(c, slot, bl + off, c->nlist_far[slot][7], o, s); off += c->nlist_far[slot][7];
    launch_vkfar<OP, 8>(c, slot, bl + off, c->nlist_far[slot][8], o, s);
    HIPCHK(c, hipGetLastError());
    return 0;
}

// Block lists: the generic kernel takes touching blocks, closed-form
// fallbacks and orders above 8; the far kernels take the rest.
int build_block_lists(stbem_ctx* c)
{
    Geom g;
    g.ng = c->ng; g.nt = c->nt; g.alpha = c->alpha; g.t = c->t.data();
    g.vx = c->vx.data(); g.vy = c->vy.data(); g.ex = c->ex.data(); g.ey = c->ey.data(); g.len = c->len.data();
    const int ops[5] = {OP_V, OP_K, OP_D, OP_DV, OP_DK}, slots[5] = {0, 1, 2, 4, 5};
    std::vector<int> far_lists[2];        // separated blocks of V_h and D_h
    TimeBlock tb;
    for (int e = 0; e < 5; ++e) {
        const int op = ops[e], slot = slots[e];
        std::vector<int> touch, gen, far[9], nterm_far[9];
        for (int k = 0; k < c->nt; ++k)
            for (int m = 0; m <= (c->toep ? 0 : k); ++m) {
                int b = (int)((long long)k * (k + 1) / 2 + m);
                time_block(g, k, m, tb);
                int q = q_block(op, c->lmax, block_min_lag(g.t, k, m), g.alpha);
                if ((op == OP_V || op == OP_D || op == OP_K || op == OP_DK) && tb.d <= 1) touch.push_back(b);
                else if (!tb.ser) gen.push_back(b);
                else if (q >= 3 && q <= 8) { far[q].push_back(b); nterm_far[q].push_back(tb.nterm); }
                else gen.push_back(b);
            }
        std::vector<int> all(touch);
        all.insert(all.end(), gen.begin(), gen.end());
        c->list_nterm[slot].assign(all.size(), 0);
        for (int q = 0; q < 9; ++q) {
            all.insert(all.end(), far[q].begin(), far[q].end());
            c->list_nterm[slot].insert(c->list_nterm[slot].end(), nterm_far[q].begin(), nterm_far[q].end());
            c->nlist_far[slot][q] = (int)far[q].size();
        }
        c->nlist_touch[slot] = (int)touch.size();
        c->nlist_gen[slot] = (int)gen.size();
        c->h_blist[slot] = all;
        int rc = upload(c, &c->d_blist[slot], all);
        if (rc) return rc;
        if (slot == 0 || slot == 2) far_lists[slot / 2].assign(all.end() - (all.size() - touch.size() - gen.size()), all.end());
    }
    c->vd_fusable = far_lists[0] == far_lists[1] && c->nlist_touch[0] == c->nlist_touch[2];
    for (int q = 0; q < 9; ++q) c->vd_fusable = c->vd_fusable && c->nlist_far[0][q] == c->nlist_far[2][q];
    {
        std::vector<char> in_dfar((size_t)c->nblk + 1, 0);      // by packed index
        std::vector<int> rest;
        for (int b : far_lists[1]) in_dfar[(size_t)b] = 1;
        const std::vector<int>& kl = c->h_blist[1];
        for (size_t e = (size_t)c->nlist_touch[1]; e < kl.size(); ++e)
            if (!in_dfar[(size_t)kl[e]]) rest.push_back(kl[e]);
        c->nklist_fused = (int)rest.size();
        if (rest.empty()) rest.push_back(0);
        int rc = upload(c, &c->d_klist_fused, rest);
        if (rc) return rc;
    }
    return 0;
}

// M0 rows k >= m0_ksplit from the power moments (k_m0_pow, _gather, _apply)
int m0_power_rows(stbem_ctx* c, bool deriv, double* o, hipStream_t s)
{
    const int npow = c->m0_npow;
    const long long per_i = (long long)npow * c->ntri * 3 * (long long)sizeof(double);
    long long ni = (1LL << 30) / (per_i > 0 ? per_i : 1);
    ni = ni < 1 ? 1 : (ni > c->ng ? c->ng : ni);
    double* S = (double*)dev_alloc(c, (size_t)(ni * per_i));
    double* G = (double*)dev_alloc(c, (size_t)c->ng * npow * c->nv * sizeof(double));
    if (!S || !G) {
        dev_free(c, S); dev_free(c, G);
        return fail(c, STBEM_ENOMEM, "M0 power-moment buffers");
    }
    Geom g = geom(c);
    int rc = 0;
    for (int i0 = 0; i0 < c->ng && !rc; i0 += (int)ni) {
        const int n = (int)std::min<long long>(ni, c->ng - i0);
        const long long lanes = (long long)n * c->ntri * 3, glanes = (long long)n * npow * c->nv;
        {
            KTimer kt(c, "k_m0_pow", (double)n * c->ntri, s);
            hipLaunchKernelGGL(k_m0_pow, dim3((unsigned)((lanes + kWG - 1) / kWG)), dim3(kWG), 0, s, g, mesh(c), c->d_tab,
                               c->m0ord.omax, c->t[c->m0_ksplit], i0, n, npow, S);
        }
        {
            KTimer kt(c, "k_m0_pow_gather", (double)n * npow * c->nv, s);
            hipLaunchKernelGGL(k_m0_pow_gather, dim3((unsigned)((glanes + kWG - 1) / kWG)), dim3(kWG), 0, s, mesh(c),
                               (const int*)c->d_v2t_loc, i0, n, npow, (const double*)S, G);
        }
        if (hipGetLastError() != hipSuccess) rc = fail(c, STBEM_EHIP, "M0 power-moment kernels");
    }
    if (!rc) {
        const long long lanes = (long long)c->ng * c->nv;
        const double sc = (deriv ? 1.0 : c->alpha) * kInv4Pi;
        KTimer kt(c, "k_m0_pow_apply", (double)(c->nt - c->m0_ksplit) * lanes, s);
        hipLaunchKernelGGL(k_m0_pow_apply, dim3((unsigned)((lanes + kWG - 1) / kWG)), dim3(kWG), 0, s, c->ng, c->nv, c->nt,
                           c->m0_ksplit, npow, (const double*)(deriv ? c->d_m0cd : c->d_m0c), sc, (const double*)G, o);
        if (hipGetLastError() != hipSuccess) rc = fail(c, STBEM_EHIP, "M0 power-moment contraction");
    }
    (void)hipStreamSynchronize(s);
    dev_free(c, S);
    dev_free(c, G);
    return rc;
}

void free_f32(stbem_ctx* c, bool v, bool d)
{
    if (v) { dev_free(c, c->v_hi); dev_free(c, c->v_lo); c->v_hi = c->v_lo = nullptr; }
    if (d) { dev_free(c, c->d_32); c->d_32 = nullptr; }
}

void free_slot(stbem_ctx* c, int slot)
{
    dev_free(c, c->mat[slot]);
    c->mat[slot] = nullptr;
    c->mat_bytes[slot] = 0;
}

// where the kernels write operator `slot` (V_h: FP64, or the hi + lo pair;
// D_h: FP64 or FP32; the others FP64)
OutBuf out_of(const stbem_ctx* c, int slot)
{
    if (slot == 0 && !c->mat[0]) return OutBuf{nullptr, c->v_hi, c->v_lo};
    if (slot == 2 && !c->mat[2]) return OutBuf{nullptr, c->d_32, nullptr};
    return OutBuf{c->mat[slot], nullptr, nullptr};
}

// Storage for one operator before its kernels run.  FP64: the FP64 array;
// FP32 copies of V_h or D_h made earlier would be stale and are freed.
// FP32_IR (V_h, D_h only): V_h as the pair hi + lo, D_h as FP32; the FP64
// array of the operator is freed.
int prepare_storage(stbem_ctx* c, unsigned op, int prec)
{
    const int slot = op_slot(op);
    if (prec == STBEM_FP32_IR) {
        const size_t fb = (size_t)causal_entries(c) * sizeof(float);
        free_slot(c, slot);
        if (op == STBEM_V) {
            if (!c->v_hi) c->v_hi = (float*)dev_alloc(c, fb);
            if (!c->v_lo) c->v_lo = (float*)dev_alloc(c, fb);
            if (!c->v_hi || !c->v_lo) { free_f32(c, true, false); return fail(c, STBEM_ENOMEM, "FP32 storage of V_h (2 x %zu bytes)", fb); }
        } else {
            if (!c->d_32) c->d_32 = (float*)dev_alloc(c, fb);
            if (!c->d_32) return fail(c, STBEM_ENOMEM, "FP32 storage of D_h (%zu bytes)", fb);
        }
        return 0;
    }
    size_t bytes = (op == STBEM_M0 || op == STBEM_DM0) ? (size_t)c->n * c->nv * sizeof(double)
                                                      : (size_t)causal_entries(c) * sizeof(double);
    if ((op == STBEM_M0 || op == STBEM_DM0) && c->nv == 0) return fail(c, STBEM_EINVAL, "no Omega mesh for M0");
    if (op == STBEM_V || op == STBEM_D) free_f32(c, op == STBEM_V, op == STBEM_D);
    if (c->mat[slot] && c->mat_bytes[slot] != bytes) free_slot(c, slot);
    if (!c->mat[slot]) {
        c->mat[slot] = (double*)dev_alloc(c, bytes);
        if (!c->mat[slot]) return fail(c, STBEM_ENOMEM, "allocation of %zu bytes for operator %u failed", bytes, op);
        c->mat_bytes[slot] = bytes;
    }
    return 0;
}

// D_h's separated blocks in FP32 arithmetic into FP32 storage (the float
// series table is built on first use)
int launch_dfar32(stbem_ctx* c, const int* bl, OutBuf od, hipStream_t s)
{
    if (!c->d_tbs32) {
        if (hipMalloc((void**)&c->d_tbs32, (size_t)c->nblk * sizeof(TimeBlock32)) != hipSuccess) {
            (void)hipGetLastError();
            c->d_tbs32 = nullptr;
            return fail(c, STBEM_ENOMEM, "float series table (%zu bytes)", (size_t)c->nblk * sizeof(TimeBlock32));
        }
        hipLaunchKernelGGL(k_time_blocks32, dim3((unsigned)((c->nblk + kWG - 1) / kWG)), dim3(kWG), 0, s, geom(c), c->nblk,
                           c->d_tbs32);
        HIPCHK(c, hipGetLastError());
    }
    const int t1 = (c->ng + kTile - 1) / kTile;
    const long long tiles = tiles_per_block(t1, true);
    const int step = blocks_per_launch(tiles);
    // The blocks of the FP64 rule q take q - 1 points per direction: the FP32
    // entries need about 1e-7 of the block maximum, which the shorter rule
    // still meets (the FP64 orders are set for 1e-15).
    for (int q = 3; q <= 8; ++q) {
        for (int off = 0; off < c->nlist_far[2][q]; off += step) {
            const int n = std::min(step, c->nlist_far[2][q] - off);
            dim3 gr((unsigned)(n * tiles)), blk(kWG);
            const int* b2 = bl + off;
            KTimer kt(c, (std::string("k_assemble_dfar32<") + std::to_string(q - 1) + ">").c_str(), (double)n * c->ng * c->ng, s);
            switch (q) {
            case 3: hipLaunchKernelGGL((k_assemble_dfar32<2>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            case 4: hipLaunchKernelGGL((k_assemble_dfar32<3>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            case 5: hipLaunchKernelGGL((k_assemble_dfar32<4>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            case 6: hipLaunchKernelGGL((k_assemble_dfar32<5>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            case 7: hipLaunchKernelGGL((k_assemble_dfar32<6>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            default: hipLaunchKernelGGL((k_assemble_dfar32<7>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, c->d_tbs32); break;
            }
        }
        bl += c->nlist_far[2][q];
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

int assemble_one(stbem_ctx* c, unsigned op, hipStream_t s, bool fuse_vd, int prec, bool fuse_k = false)
{
    int slot = op_slot(op);
    int rc0 = prepare_storage(c, op, prec);
    if (rc0) return rc0;
    double* o = c->mat[slot];
    switch (op) {
    case STBEM_V:
    case STBEM_K: {
        if (op == STBEM_K) launch_knear<OP_K>(c, 1, o, s);
        const OutBuf ob = out_of(c, slot);
        // K_h with V_h and D_h: its separated blocks in D_h's far lists come
        // from D_h's far tiles, the generic kernel takes the rest
        if (op == STBEM_K && fuse_k) return launch_assemble_list<OP_K>(c, ob, s, c->d_klist_fused, c->nklist_fused);
        // V_h with D_h: its touching and separated blocks come with D_h's tiles
        int rc = op == STBEM_V ? launch_assemble<OP_V>(c, ob, s, !fuse_vd) : launch_assemble<OP_K>(c, ob, s);
        if (rc) return rc;
        // fused with D_h in FP64; in the FP32-storage mode D_h's far field is
        // computed in FP32 by its own tiles, V_h's (which the refinement
        // residual needs to FP64 accuracy) by the FP64 far tiles
        if (op == STBEM_V && fuse_vd && prec != STBEM_FP32_IR) return 0;
        return op == STBEM_V ? launch_far<OP_V>(c, 0, ob, s) : launch_far<OP_K>(c, 1, ob, s);
    }
    case STBEM_D: {
        const OutBuf od = out_of(c, 2), ov = out_of(c, 0);
        int t1 = (c->ng + kTile - 1) / kTile;
        const long long tiles = tiles_per_block(t1, true);
        const int step = blocks_per_launch(tiles);
        for (int off = 0; off < c->nlist_touch[2]; off += step) {
            const int n = std::min(step, c->nlist_touch[2] - off);
            KTimer kt(c, store_name(fuse_vd ? "k_assemble_dnear<true>" : "k_assemble_dnear<false>", od).c_str(),
                      (double)n * c->ng * c->ng, s);
            if (fuse_vd)
                hipLaunchKernelGGL(k_assemble_dnear<true>, dim3((unsigned)(n * tiles)), dim3(kWG), 0, s, geom(c), c->d_tab, c->ord,
                                   (const int*)(c->d_blist[2] + off), t1, od, ov);
            else
                hipLaunchKernelGGL(k_assemble_dnear<false>, dim3((unsigned)(n * tiles)), dim3(kWG), 0, s, geom(c), c->d_tab, c->ord,
                                   (const int*)(c->d_blist[2] + off), t1, od, OutBuf{nullptr, nullptr, nullptr});
        }
        int rc = launch_assemble<OP_D>(c, od, s);
        if (rc) return rc;
        const int* bl = c->d_blist[2] + c->nlist_touch[2] + c->nlist_gen[2];
        const OutBuf none{nullptr, nullptr, nullptr};
        if (prec == STBEM_FP32_IR) return launch_dfar32(c, bl, od, s);
        for (int q = 3; q <= 8; ++q) {
            for (int off = 0; off < c->nlist_far[2][q]; off += step) {
                const int n = std::min(step, c->nlist_far[2][q] - off);
                dim3 gr((unsigned)(n * tiles)), blk(kWG);
                const int* b2 = bl + off;
                const std::string kn = std::string("k_assemble_dfar<") + std::to_string(q) +
                                       (fuse_vd ? (fuse_k ? ", true, true>" : ", true>") : ", false>");
                KTimer kt(c, store_name(kn.c_str(), od).c_str(), (double)n * c->ng * c->ng, s,
                          c->timing ? flops_dfar(q, fuse_vd, n, sum_terms(c, 2, b2, n), tiles, (long long)c->ng * (c->ng + 1) / 2,
                                                 fuse_k) : 0.0);
                double* ok = c->mat[1];
                if (fuse_vd && fuse_k) switch (q) {
                case 3: hipLaunchKernelGGL((k_assemble_dfar<3, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                case 4: hipLaunchKernelGGL((k_assemble_dfar<4, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                case 5: hipLaunchKernelGGL((k_assemble_dfar<5, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                case 6: hipLaunchKernelGGL((k_assemble_dfar<6, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                case 7: hipLaunchKernelGGL((k_assemble_dfar<7, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                default: hipLaunchKernelGGL((k_assemble_dfar<8, true, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs, ok); break;
                }
                else if (fuse_vd) switch (q) {
                case 3: hipLaunchKernelGGL((k_assemble_dfar<3, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                case 4: hipLaunchKernelGGL((k_assemble_dfar<4, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                case 5: hipLaunchKernelGGL((k_assemble_dfar<5, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                case 6: hipLaunchKernelGGL((k_assemble_dfar<6, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                case 7: hipLaunchKernelGGL((k_assemble_dfar<7, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                default: hipLaunchKernelGGL((k_assemble_dfar<8, true>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, ov, c->d_tbs); break;
                }
                else switch (q) {
                case 3: hipLaunchKernelGGL((k_assemble_dfar<3, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                case 4: hipLaunchKernelGGL((k_assemble_dfar<4, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                case 5: hipLaunchKernelGGL((k_assemble_dfar<5, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                case 6: hipLaunchKernelGGL((k_assemble_dfar<6, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                case 7: hipLaunchKernelGGL((k_assemble_dfar<7, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                default: hipLaunchKernelGGL((k_assemble_dfar<8, false>), gr, blk, 0, s, geom(c), c->d_tab, b2, t1, od, none, c->d_tbs); break;
                }
            }
            bl += c->nlist_far[2][q];
        }
        HIPCHK(c, hipGetLastError());
        return 0;
    }
    case STBEM_DV: {
        int rc = launch_assemble<OP_DV>(c, out_of(c, 4), s);
        return rc ? rc : launch_far<OP_DV>(c, 4, out_of(c, 4), s);
    }
    case STBEM_DK: {
        launch_knear<OP_DK>(c, 5, o, s);
        int rc = launch_assemble<OP_DK>(c, out_of(c, 5), s);
        return rc ? rc : launch_far<OP_DK>(c, 5, out_of(c, 5), s);
    }
    case STBEM_M0:
    case STBEM_DM0: {
        // whole time rows in chunks whose moment scratch stays below 1 GiB:
        // the first time element by the per-row kernel with the singular
        // rules, the later rows below the power-series split by k_m0_rows
        long long per_row = (long long)c->ntri * 3 * (long long)sizeof(double);
        long long krows = (1LL << 30) / (per_row * c->ng > 0 ? per_row * c->ng : 1);
        krows = krows < 1 ? 1 : (krows > c->m0_ksplit ? (c->m0_ksplit > 0 ? c->m0_ksplit : 1) : krows);
        double* scratch = (double*)dev_alloc(c, (size_t)(krows * c->ng * per_row));
        if (!scratch) return fail(c, STBEM_ENOMEM, "M0 scratch of %lld bytes", krows * c->ng * per_row);
        int tchunk = (c->ntri + kWG - 1) / kWG, vchunk = (c->nv + kWG - 1) / kWG;
        int rc = 0;
        for (int kc0 = 0; kc0 < c->m0_ksplit && !rc; kc0 += (int)krows) {
            const int kc1 = (int)std::min<long long>(kc0 + krows, c->m0_ksplit);
            const long long r0 = (long long)kc0 * c->ng, nr = (long long)(kc1 - kc0) * c->ng;
            if (kc0 == 0) {
                // the first time element in two launches: the pairs with the
                // regular rule (few registers), then the near pairs
                const dim3 gr((unsigned)(c->ng * tchunk));
                {
                    KTimer kt(c, op == STBEM_M0 ? "k_m0_tri<false, true, 1>" : "k_m0_tri<true, true, 1>", (double)c->ng * c->ntri, s);
                    if (op == STBEM_M0)
                        hipLaunchKernelGGL((k_m0_tri<false, true, 1>), gr, dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->d_m0tab, c->m0ord, m0poly(c), 0LL, 0LL, tchunk, scratch);
                    else
                        hipLaunchKernelGGL((k_m0_tri<true, true, 1>), gr, dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->d_m0tab, c->m0ord, m0poly(c), 0LL, 0LL, tchunk, scratch);
                }
                KTimer kt(c, op == STBEM_M0 ? "k_m0_tri<false, true, 2>" : "k_m0_tri<true, true, 2>", (double)c->ng * c->ntri, s);
                if (op == STBEM_M0)
                    hipLaunchKernelGGL((k_m0_tri<false, true, 2>), gr, dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->d_m0tab, c->m0ord, m0poly(c), 0LL, 0LL, tchunk, scratch);
                else
                    hipLaunchKernelGGL((k_m0_tri<true, true, 2>), gr, dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->d_m0tab, c->m0ord, m0poly(c), 0LL, 0LL, tchunk, scratch);
            }
            const int k0 = kc0 > 0 ? kc0 : 1;
            if (k0 < kc1) {
                KTimer kt(c, op == STBEM_M0 ? "k_m0_rows<false>" : "k_m0_rows<true>", (double)(kc1 - k0) * c->ng * c->ntri, s);
                if (op == STBEM_M0)
                    hipLaunchKernelGGL((k_m0_rows<false>), dim3((unsigned)(c->ng * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->m0ord, m0poly(c), r0, k0, kc1 - k0, tchunk, scratch);
                else
                    hipLaunchKernelGGL((k_m0_rows<true>), dim3((unsigned)(c->ng * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->m0ord, m0poly(c), r0, k0, kc1 - k0, tchunk, scratch);
            }
            KTimer kt(c, "k_m0_gather", (double)nr * c->nv, s);
            hipLaunchKernelGGL(k_m0_gather, dim3((unsigned)(nr * vchunk)), dim3(kWG), 0, s, mesh(c), (const int*)c->d_v2t_loc, r0, vchunk, (const double*)scratch, o);
            if (hipGetLastError() != hipSuccess) rc = fail(c, STBEM_EHIP, "M0 kernels");
        }
        (void)hipStreamSynchronize(s);
        dev_free(c, scratch);
        if (!rc && c->m0_ksplit < c->nt) rc = m0_power_rows(c, op == STBEM_DM0, o, s);
        return rc;
    }
    }
    return fail(c, STBEM_EINVAL, "unknown operator %u", op);
}

// y = A x (A^T x) for block-Toeplitz storage A_d = block (m + d, m): one
// launch of k_toeplitz_mfma over the 64 x 64 tiles of Y.
int toeplitz_apply(stbem_ctx* c, const double* A, int trans, const double* x, double* y, hipStream_t s)
{
    const int ng = c->ng, nt = c->nt;
    const int tr = (ng + kTT - 1) / kTT, tc = (nt + kTT - 1) / kTT;
    const int ntile = tr * tc, grid = 8 * ((ntile + 7) / 8);
    const bool vec = ng % 16 == 0 && ((uintptr_t)A % 32) == 0 && ((uintptr_t)x % 32) == 0;
    KTimer kt(c, trans ? "k_toeplitz_mfma<1>" : "k_toeplitz_mfma<0>", (double)causal_entries(c), s);
    if (!trans) {
        if (vec) hipLaunchKernelGGL((k_toeplitz_mfma<0, true>), dim3(grid), dim3(kWG), 0, s, A, x, y, ng, nt, tr, tc);
        else hipLaunchKernelGGL((k_toeplitz_mfma<0, false>), dim3(grid), dim3(kWG), 0, s, A, x, y, ng, nt, tr, tc);
    } else {
        if (vec) hipLaunchKernelGGL((k_toeplitz_mfma<1, true>), dim3(grid), dim3(kWG), 0, s, A, x, y, ng, nt, tr, tc);
        else hipLaunchKernelGGL((k_toeplitz_mfma<1, false>), dim3(grid), dim3(kWG), 0, s, A, x, y, ng, nt, tr, tc);
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

// Pass 1 of y = A x (A^T x) for packed causal storage (FP64, or hi+lo FP32
// pair, or FP32): the partial vectors of the packed blocks [b0, b0 + nb)
// into part[(b - b0) * ng + i].
int gemv_partials(stbem_ctx* c, const double* A, const float* hi, const float* lo, const float* a32, int trans,
                  const double* x, double* part, long long b0, long long nb, hipStream_t s)
{
    const int ng = c->ng;
    // vector width: the row length must be a multiple of 64 * VW
    const int vw64 = (ng % 128 == 0) ? 2 : 1;
    const int vw32 = (ng % 256 == 0) ? 4 : (ng % 128 == 0 ? 2 : 1);
    if (!trans) {
        int rowchunks = (ng + 4 * kRowsPerWave - 1) / (4 * kRowsPerWave);
        dim3 gr((unsigned)(nb * rowchunks)), bl(kWG);
        if (A) {
            if (vw64 == 2) hipLaunchKernelGGL((k_gemv_n_vec<double, 2, double, false, 2>), gr, bl, 0, s, A, (const double*)nullptr, x, part, ng, rowchunks, b0);
            else hipLaunchKernelGGL((k_gemv_n_vec<double, 1, double, false>), gr, bl, 0, s, A, (const double*)nullptr, x, part, ng, rowchunks, b0);
        } else if (hi) {
            if (vw32 == 4) hipLaunchKernelGGL((k_gemv_n_vec<float, 4, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, rowchunks, b0);
            else if (vw32 == 2) hipLaunchKernelGGL((k_gemv_n_vec<float, 2, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, rowchunks, b0);
            else hipLaunchKernelGGL((k_gemv_n_vec<float, 1, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, rowchunks, b0);
        } else {
            if (vw32 == 4) hipLaunchKernelGGL((k_gemv_n_vec<float, 4, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, rowchunks, b0);
            else if (vw32 == 2) hipLaunchKernelGGL((k_gemv_n_vec<float, 2, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, rowchunks, b0);
            else hipLaunchKernelGGL((k_gemv_n_vec<float, 1, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, rowchunks, b0);
        }
    } else {
        if (A) {
            int cc = (ng + 64 * vw64 - 1) / (64 * vw64);
            dim3 gr((unsigned)(nb * cc)), bl(kWG);
            if (vw64 == 2) hipLaunchKernelGGL((k_gemv_t_vec<double, 2, double, false>), gr, bl, 0, s, A, (const double*)nullptr, x, part, ng, cc, b0);
            else hipLaunchKernelGGL((k_gemv_t_vec<double, 1, double, false>), gr, bl, 0, s, A, (const double*)nullptr, x, part, ng, cc, b0);
        } else {
            int cc = (ng + 64 * vw32 - 1) / (64 * vw32);
            dim3 gr((unsigned)(nb * cc)), bl(kWG);
            if (hi) {
                if (vw32 == 4) hipLaunchKernelGGL((k_gemv_t_vec<float, 4, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, cc, b0);
                else if (vw32 == 2) hipLaunchKernelGGL((k_gemv_t_vec<float, 2, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, cc, b0);
                else hipLaunchKernelGGL((k_gemv_t_vec<float, 1, double, true>), gr, bl, 0, s, hi, lo, x, part, ng, cc, b0);
            } else {
                if (vw32 == 4) hipLaunchKernelGGL((k_gemv_t_vec<float, 4, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, cc, b0);
                else if (vw32 == 2) hipLaunchKernelGGL((k_gemv_t_vec<float, 2, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, cc, b0);
                else hipLaunchKernelGGL((k_gemv_t_vec<float, 1, float, false>), gr, bl, 0, s, a32, (const float*)nullptr, x, part, ng, cc, b0);
            }
        }
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

// Pass 2: the outputs of the block rows [k0, k1) (trans: the block columns
// [0, k1), accumulated over row ranges) from their partials.
int gemv_reduce(stbem_ctx* c, const double* part, double* y, int trans, int k0, int k1, hipStream_t s)
{
    const long long outs = (long long)(trans ? k1 : k1 - k0) * c->ng;
    const long long pb0 = (long long)k0 * (k0 + 1) / 2;
    hipLaunchKernelGGL(k_gemv_reduce, dim3((unsigned)((outs + kRedOut - 1) / kRedOut)), dim3(kWG), 0, s, part, y, c->ng,
                       k0, k1, pb0, trans);
    HIPCHK(c, hipGetLastError());
    return 0;
}

const char* gemv_name(const double* A, const float* hi, int trans)
{
    return !trans ? (A ? "k_gemv_n_vec<double>" : hi ? "k_gemv_n_vec<float hi+lo>" : "k_gemv_n_vec<float>")
                  : (A ? "k_gemv_t_vec<double>" : hi ? "k_gemv_t_vec<float hi+lo>" : "k_gemv_t_vec<float>");
}

// y = A x for packed causal storage (FP64, or hi+lo FP32 pair, or FP32)
int packed_apply(stbem_ctx* c, const double* A, const float* hi, const float* lo, const float* a32, int trans,
                 const double* x, double* y, hipStream_t s)
{
    if (c->toep) {
        if (!A) return fail(c, STBEM_EINVAL, "FP32 products need packed storage (block-Toeplitz mode is FP64 only)");
        return toeplitz_apply(c, A, trans, x, y, s);
    }
    int rc = ensure_part(c);
    if (rc) return rc;
    {
        KTimer kt(c, gemv_name(A, hi, trans), (double)c->nblk * c->ng * c->ng, s);
        if ((rc = gemv_partials(c, A, hi, lo, a32, trans, x, c->part, 0, c->nblk, s))) return rc;
    }
    return gemv_reduce(c, c->part, y, trans, 0, c->nt, s);
}

int dense_apply(stbem_ctx* c, const double* M, int trans, const double* x, double* y, hipStream_t s)
{
    if (!trans) {
        hipLaunchKernelGGL(k_dense_n, dim3((unsigned)((c->n + 3) / 4)), dim3(kWG), 0, s, M, x, y, c->n, c->nv);
    } else {
        int rc = ensure_part(c);
        if (rc) return rc;
        int nrc = (int)((c->n + 255) / 256), colchunks = (c->nv + kWG - 1) / kWG;
        hipLaunchKernelGGL(k_dense_t_part, dim3((unsigned)((long long)nrc * colchunks)), dim3(kWG), 0, s, M, x, c->part, c->n, c->nv, colchunks);
        hipLaunchKernelGGL(k_dense_t_reduce, dim3((unsigned)colchunks), dim3(kWG), 0, s, c->part, y, nrc, c->nv);
    }
    HIPCHK(c, hipGetLastError());
    return 0;
}

// y = M_h^0 u0 without storing M_h^0 (for meshes where the N x M_Omega
// matrix does not fit): chunks of rows are computed by the per-row moment
// kernels, gathered into a chunk buffer and applied, in row order.
int m0_fused_apply(stbem_ctx* c, const double* u0, double* y, hipStream_t s, bool deriv = false)
{
    if (c->nv == 0) return fail(c, STBEM_EINVAL, "no Omega mesh for M0");
    const long long per_row = (long long)c->ntri * 3 * (long long)sizeof(double) + (long long)c->nv * sizeof(double);
    long long rows = (1LL << 30) / per_row;
    rows = rows < 1 ? 1 : (rows > c->n ? c->n : rows);
    double* scratch = (double*)dev_alloc(c, (size_t)(rows * c->ntri * 3 * sizeof(double)));
    double* buf = (double*)dev_alloc(c, (size_t)(rows * c->nv * sizeof(double)));
    if (!scratch || !buf) {
        dev_free(c, scratch); dev_free(c, buf);
        return fail(c, STBEM_ENOMEM, "M0 chunk buffers");
    }
    const int tchunk = (c->ntri + kWG - 1) / kWG, vchunk = (c->nv + kWG - 1) / kWG;
    int rc = 0;
    for (long long r0 = 0; r0 < c->n && !rc; r0 += rows) {
        const long long nr = std::min(rows, c->n - r0);
        const long long nf = r0 < c->ng ? std::min<long long>(nr, c->ng - r0) : 0, nl = nr - nf;
        if (nf > 0) {
            KTimer kt(c, deriv ? "k_m0_tri<true, true>" : "k_m0_tri<false, true>", (double)nf * c->ntri, s);
            if (deriv)
                hipLaunchKernelGGL((k_m0_tri<true, true>), dim3((unsigned)(nf * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab,
                                   c->d_m0tab, c->m0ord, m0poly(c), r0, 0LL, tchunk, scratch);
            else
                hipLaunchKernelGGL((k_m0_tri<false, true>), dim3((unsigned)(nf * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab,
                                   c->d_m0tab, c->m0ord, m0poly(c), r0, 0LL, tchunk, scratch);
        }
        if (nl > 0) {
            KTimer kt(c, deriv ? "k_m0_tri<true, false>" : "k_m0_tri<false, false>", (double)nl * c->ntri, s);
            if (deriv)
                hipLaunchKernelGGL((k_m0_tri<true, false>), dim3((unsigned)(nl * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab,
                                   c->d_m0tab, c->m0ord, m0poly(c), r0, nf, tchunk, scratch);
            else
                hipLaunchKernelGGL((k_m0_tri<false, false>), dim3((unsigned)(nl * tchunk)), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab,
                                   c->d_m0tab, c->m0ord, m0poly(c), r0, nf, tchunk, scratch);
        }
        hipLaunchKernelGGL(k_m0_gather, dim3((unsigned)(nr * vchunk)), dim3(kWG), 0, s, mesh(c), (const int*)c->d_v2t_loc, 0LL,
                           vchunk, (const double*)scratch, buf);
        hipLaunchKernelGGL(k_dense_n, dim3((unsigned)((nr + 3) / 4)), dim3(kWG), 0, s, (const double*)buf, u0, y + r0, nr, c->nv);
        if (hipGetLastError() != hipSuccess) rc = fail(c, STBEM_EHIP, "fused M0 kernels");
    }
    (void)hipStreamSynchronize(s);
    dev_free(c, scratch);
    dev_free(c, buf);
    return rc;
}

// y = A x for A = dV_h/dalpha (slot 4) or dK_h/dalpha (slot 5) without
// storing A: the block rows are assembled in ranges into a bounded buffer
// (<= 1 GiB, at least one block row) by the same kernels as the stored
// operator, and each range is contracted with x right away (the same two
// GEMV passes); y's block rows [k0, k1) are final after their range.  The
// block lists of the slot are swapped for the range's sub-lists (each list
// group is in increasing k, so a range keeps the group structure).
int deriv_apply_blockwise(stbem_ctx* c, int slot, const double* x, double* y, hipStream_t s)
{
    if (c->toep) return fail(c, STBEM_ENOTASSEMBLED, "alpha-derivative operators not assembled (block-Toeplitz mode)");
    const long long ng2 = (long long)c->ng * c->ng;
    long long cap = (1LL << 30) / (ng2 * (long long)sizeof(double));
    if (cap < c->nt) cap = c->nt;
    if (cap > c->nblk) cap = c->nblk;
    int rc = ensure_part(c);
    if (rc) return rc;
    const std::vector<int>& all = c->h_blist[slot];
    double* T = (double*)dev_alloc(c, (size_t)(cap * ng2 * (long long)sizeof(double)));
    int* dl = (int*)dev_alloc(c, (all.empty() ? 1 : all.size()) * sizeof(int));
    if (!T || !dl) {
        dev_free(c, T); dev_free(c, dl);
        return fail(c, STBEM_ENOMEM, "blockwise alpha-derivative buffers (%lld blocks)", cap);
    }
    // list groups: touch | gen | far Q = 3..8
    int gsz[8] = {c->nlist_touch[slot], c->nlist_gen[slot]};
    for (int q = 3; q <= 8; ++q) gsz[q - 1] = c->nlist_far[slot][q];
    int* const save_list = c->d_blist[slot];
    const int save_touch = c->nlist_touch[slot], save_gen = c->nlist_gen[slot];
    int save_far[9];
    for (int q = 0; q < 9; ++q) save_far[q] = c->nlist_far[slot][q];
    std::vector<int> save_nterm = c->list_nterm[slot];
    auto row_of = [](long long b) { long long k = (long long)((std::sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
                                    while (k * (k + 1) / 2 > b) --k;
                                    while ((k + 1) * (k + 2) / 2 <= b) ++k;
                                    return (int)k; };
    for (int k0 = 0; k0 < c->nt && !rc; ) {
        const long long pb0 = (long long)k0 * (k0 + 1) / 2;
        int k1 = k0 + 1;
        while (k1 < c->nt && (long long)(k1 + 1) * (k1 + 2) / 2 - pb0 <= cap) ++k1;
        std::vector<int> sub, subn;
        int cnt[8];
        int at = 0;
        for (int gi = 0; gi < 8; ++gi) {
            cnt[gi] = 0;
            for (int e = at; e < at + gsz[gi]; ++e) {
                const int kb = row_of(all[e]);
                if (kb >= k0 && kb < k1) { sub.push_back(all[e]); subn.push_back(save_nterm[e]); ++cnt[gi]; }
            }
            at += gsz[gi];
        }
        // the previous range's kernels must be done with dl and T
        if (hipStreamSynchronize(s) != hipSuccess ||
            (!sub.empty() && hipMemcpy(dl, sub.data(), sub.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)) {
            rc = fail(c, STBEM_EHIP, "blockwise alpha-derivative list upload");
            break;
        }
        c->d_blist[slot] = dl;
        c->nlist_touch[slot] = cnt[0];
        c->nlist_gen[slot] = cnt[1];
        for (int q = 3; q <= 8; ++q) c->nlist_far[slot][q] = cnt[q - 1];
        c->list_nterm[slot] = subn;
        // block b of the range is written at T + (b - pb0) ng^2
        double* Tb = (double*)((uintptr_t)T - (uintptr_t)(pb0 * ng2 * (long long)sizeof(double)));
        const OutBuf o{Tb, nullptr, nullptr};
        if (slot == 4) {
            rc = launch_assemble<OP_DV>(c, o, s);
            if (!rc) rc = launch_far<OP_DV>(c, 4, o, s);
        } else {
            launch_knear<OP_DK>(c, 5, Tb, s);
            rc = launch_assemble<OP_DK>(c, o, s);
            if (!rc) rc = launch_far<OP_DK>(c, 5, o, s);
        }
        const long long nb = (long long)k1 * (k1 + 1) / 2 - pb0;
        if (!rc) rc = gemv_partials(c, Tb, nullptr, nullptr, nullptr, 0, x, c->part, pb0, nb, s);
        if (!rc) rc = gemv_reduce(c, c->part, y, 0, k0, k1, s);
        k0 = k1;
    }
    (void)hipStreamSynchronize(s);
    c->d_blist[slot] = save_list;
    c->nlist_touch[slot] = save_touch;
    c->nlist_gen[slot] = save_gen;
    for (int q = 0; q < 9; ++q) c->nlist_far[slot][q] = save_far[q];
    c->list_nterm[slot] = save_nterm;
    dev_free(c, T);
    dev_free(c, dl);
    return rc;
}

// dot products of the nq vectors Q_q (stride ldq) with v, into h_dev[0..nq)
struct DotWork { double* part = nullptr; int nchunk = 0; };

int dots(stbem_ctx* c, DotWork& w, const double* Q, long long ldq, int nq, const double* v, double* h_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_dots_part, dim3((unsigned)w.nchunk, (unsigned)nq), dim3(kWG), 0, s, Q, ldq, v, c->n, w.part, w.nchunk);
    hipLaunchKernelGGL(k_dots_reduce, dim3((unsigned)((nq + kWG - 1) / kWG)), dim3(kWG), 0, s, w.part, w.nchunk, nq, h_dev);
    HIPCHK(c, hipGetLastError());
    return 0;
}

// Device address of noalloc_scratch on the current device, looked up once
// per device.
constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
double* noalloc_ptr[kMaxDevices] = {};

int noalloc_setup(stbem_ctx* c)
{
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, STBEM_EHIP, "device %d beyond the table of %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p)
            return fail(c, STBEM_EHIP, "hipGetSymbolAddress(noalloc_scratch): %s", hipGetErrorString(e));
        noalloc_ptr[dev] = (double*)p;
    }
    c->noalloc = noalloc_ptr[dev];
    return 0;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* stbem_last_error(const stbem_ctx* c) { return c ? c->err.c_str() : "null context"; }

// Chebyshev economisation of sum_{j<n} c_j a^j on [0, A] (long double):
// rewritten in y = 2a/A - 1, expanded in Chebyshev polynomials of y,
// truncated where the dropped coefficients sum below tol |c_0|, and written
// back in powers of y.  Returns the number of coefficients kept, 0 if more
// than kEconMax would be needed or the double polynomial, evaluated as the
// kernels do, misses the series by more than 1e-15 of its leading term.
static int econ_poly(const long double* c, int n, long double A, long double tol, double* out)
{
    constexpr int N = kPolyMax;
    long double d[N + 1] = {}, B[N + 1] = {}, t[N + 1];
    const long double h = A / 2;
    long double hp = 1;
    for (int j = 0; j < n; ++j) {                  // a^j = h^j (y + 1)^j
        const long double cj = c[j] * hp;
        long double bin = 1;
        for (int i = 0; i <= j; ++i) {
            d[i] += cj * bin;
            bin = bin * (j - i) / (i + 1);
        }
        hp *= h;
    }
    for (int i = n - 1; i >= 0; --i) {             // Horner in the Chebyshev basis
        for (int k = 0; k <= N; ++k) t[k] = 0;
        for (int k = 0; k < N; ++k) {              // y T_0 = T_1, y T_k = (T_{k+1} + T_{k-1}) / 2
            if (k == 0) t[1] += B[0];
            else { t[k + 1] += 0.5L * B[k]; t[k - 1] += 0.5L * B[k]; }
        }
        t[0] += d[i];
        for (int k = 0; k <= N; ++k) B[k] = t[k];
    }
    int K = n;
    long double drop = 0;
    while (K > 1 && drop + fabsl(B[K - 1]) < tol * fabsl(c[0])) { drop += fabsl(B[K - 1]); --K; }
    if (K > kEconMax) return 0;
    long double P[N + 1] = {}, Tm[N + 1] = {}, Tc[N + 1] = {}, Tn[N + 1];
    Tm[0] = 1; Tc[1] = 1;
    for (int i = 0; i <= N; ++i) P[i] = B[0] * Tm[i] + (K > 1 ? B[1] * Tc[i] : 0.0L);
    for (int k = 2; k < K; ++k) {                  // T_{k} = 2 y T_{k-1} - T_{k-2}
        for (int i = 0; i <= N; ++i) Tn[i] = (i > 0 ? 2 * Tc[i - 1] : 0.0L) - Tm[i];
        for (int i = 0; i <= N; ++i) { P[i] += B[k] * Tn[i]; Tm[i] = Tc[i]; Tc[i] = Tn[i]; }
    }
    for (int i = 0; i < kEconMax; ++i) out[i] = i < K ? (double)P[i] : 0.0;
    // the double polynomial against the series, at 65 points of [0, A]
    const double es = (double)(2.0L / A);
    for (int q = 0; q <= 64; ++q) {
        const long double a = A * q / 64;
        long double ref = 0;
        for (int j = n - 1; j >= 0; --j) ref = ref * a + c[j];
        const double got = m0_econ(out, std::fma((double)a, es, -1.0));    // as the kernels evaluate it
        if (fabsl((long double)got - ref) > 1e-15L * fabsl(c[0])) return 0;
    }
    return K;
}

int stbem_create(const stbem_problem* p, stbem_ctx** out)
{
    if (!p || !out) return STBEM_EINVAL;
    *out = nullptr;
    if (!(p->alpha > 0) || !std::isfinite(p->alpha)) return STBEM_EALPHA;
    if (p->n_t < 1 || !p->t_nodes) return STBEM_ETIME;
    if (p->t_nodes[0] != 0.0) return STBEM_ETIME;
    for (int i = 0; i < p->n_t; ++i)
        if (!(p->t_nodes[i + 1] > p->t_nodes[i]) || !std::isfinite(p->t_nodes[i + 1])) return STBEM_ETIME;
    if (p->n_bnd < 3 || !p->bnd_xy) return STBEM_EMESH;
    if (p->n_vtx < 0 || p->n_tri < 0 || (p->n_vtx > 0 && (!p->vtx_xy || !p->tri || p->n_tri < 1))) return STBEM_EMESH;
    stbem_ctx* c = new stbem_ctx();
    c->ng = p->n_bnd; c->nt = p->n_t; c->nv = p->n_vtx; c->ntri = p->n_vtx > 0 ? p->n_tri : 0;
    c->alpha = p->alpha;
    c->n = (long long)c->ng * c->nt;
    c->nblk = (long long)c->nt * (c->nt + 1) / 2;
    c->packed = c->nblk * (long long)c->ng * c->ng;
    c->t.assign(p->t_nodes, p->t_nodes + c->nt + 1);
    double area2 = 0.0;
    for (int i = 0; i < c->ng; ++i) {
        double x = p->bnd_xy[2 * i], y = p->bnd_xy[2 * i + 1];
        if (!std::isfinite(x) || !std::isfinite(y)) { delete c; return STBEM_EMESH; }
        c->vx.push_back(x); c->vy.push_back(y);
    }
    for (int i = 0; i < c->ng; ++i) {
        int j = (i + 1) % c->ng;
        double dx = c->vx[j] - c->vx[i], dy = c->vy[j] - c->vy[i], L = std::sqrt(dx * dx + dy * dy);
        if (!(L > 0)) { delete c; return STBEM_EMESH; }
        c->len.push_back(L); c->ex.push_back(dx / L); c->ey.push_back(dy / L);
        area2 += c->vx[i] * c->vy[j] - c->vx[j] * c->vy[i];
        if (L > c->lmax) c->lmax = L;
    }
    if (!(area2 > 0)) { delete c; return STBEM_EMESH; }     // clockwise or degenerate
    if (c->nv > 0) {
        c->ox.resize(c->nv); c->oy.resize(c->nv);
        for (int v = 0; v < c->nv; ++v) { c->ox[v] = p->vtx_xy[2 * v]; c->oy[v] = p->vtx_xy[2 * v + 1]; }
        c->tri.assign(p->tri, p->tri + 3 * c->ntri);
        c->v2t_ptr.assign(c->nv + 1, 0);
        for (int e = 0; e < 3 * c->ntri; ++e) {
            int v = c->tri[e];
            if (v < 0 || v >= c->nv) { delete c; return STBEM_EMESH; }
            c->v2t_ptr[v + 1]++;
        }
        for (int t = 0; t < c->ntri; ++t) {
            const int* q = &c->tri[3 * t];
            double det = (c->ox[q[1]] - c->ox[q[0]]) * (c->oy[q[2]] - c->oy[q[0]]) - (c->oy[q[1]] - c->oy[q[0]]) * (c->ox[q[2]] - c->ox[q[0]]);
            if (!(det > 0)) { delete c; return STBEM_EMESH; }
        }
        for (int v = 0; v < c->nv; ++v) c->v2t_ptr[v + 1] += c->v2t_ptr[v];
        c->v2t.assign(3 * c->ntri, 0);
        c->v2t_loc.assign(3 * c->ntri, 0);
        std::vector<int> fill(c->nv, 0);
        for (int e = 0; e < 3 * c->ntri; ++e) {
            int v = c->tri[e], p = c->v2t_ptr[v] + fill[v]++;
            c->v2t[p] = e / 3;
            c->v2t_loc[p] = e % 3;
        }
    }
    // lumped dual mass Mt[(m,i)] = h_m (L_{i-1} + 2 L_i + L_{i+1}) / 4  (row sums, Sec. 4)
    std::vector<double> mt(c->n);
    for (int m = 0; m < c->nt; ++m)
        for (int i = 0; i < c->ng; ++i) {
            int im = (i + c->ng - 1) % c->ng, ip = (i + 1) % c->ng;
            mt[(long long)m * c->ng + i] = (c->t[m + 1] - c->t[m]) * (c->len[im] + 2 * c->len[i] + c->len[ip]) / 4;
        }
    int rc = 0;
    if ((rc = upload(c, &c->d_t, c->t)) || (rc = upload(c, &c->d_vx, c->vx)) || (rc = upload(c, &c->d_vy, c->vy)) ||
        (rc = upload(c, &c->d_ex, c->ex)) || (rc = upload(c, &c->d_ey, c->ey)) || (rc = upload(c, &c->d_len, c->len)) ||
        (rc = upload(c, &c->d_mt, mt)) || (rc = upload(c, &c->d_ox, c->ox)) || (rc = upload(c, &c->d_oy, c->oy)) ||
        (rc = upload(c, &c->d_tri, c->tri)) || (rc = upload(c, &c->d_v2t_ptr, c->v2t_ptr)) || (rc = upload(c, &c->d_v2t, c->v2t)) ||
        (rc = upload(c, &c->d_v2t_loc, c->v2t_loc)) || (rc = noalloc_setup(c))) {
        stbem_destroy(c);
        return rc;
    }
    Tables T;
    build_tables(T);
    M0Tables D;
    {
        // tanh-sinh on [0,1]: x = (1 + tanh(pi/2 sinh t))/2, t = -3..3, step 1/8
        const double hstep = 0.125;
        int n = 0;
        for (int q = -24; q <= 24; ++q) {
            double tt = q * hstep, u = 0.5 * M_PI * std::sinh(tt), ch = std::cosh(u);
            D.de_x[n] = 0.5 * (1.0 + std::tanh(u));
            D.de_w[n] = hstep * 0.25 * M_PI * std::cosh(tt) / (ch * ch);
            ++n;
        }
        D.nde = n;
    }
    if (hipMalloc((void**)&c->d_tab, sizeof(Tables)) != hipSuccess || hipMalloc((void**)&c->d_m0tab, sizeof(M0Tables)) != hipSuccess) {
        stbem_destroy(c);
        return STBEM_ENOMEM;
    }
    if (hipMemcpy(c->d_tab, &T, sizeof(Tables), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_m0tab, &D, sizeof(M0Tables), hipMemcpyHostToDevice) != hipSuccess) {
        stbem_destroy(c);
        return STBEM_EHIP;
    }
    c->ord = default_orders();
    {
        const long long nb = (long long)c->nt * (c->nt + 1) / 2;
        if (hipMalloc((void**)&c->d_tbs, (size_t)nb * sizeof(TimeBlock)) != hipSuccess) {
            (void)hipGetLastError();
            stbem_destroy(c);
            return STBEM_ENOMEM;
        }
        hipLaunchKernelGGL(k_time_blocks, dim3((unsigned)((nb + kWG - 1) / kWG)), dim3(kWG), 0, 0, geom(c), nb, c->d_tbs);
        if (hipDeviceSynchronize() != hipSuccess) { stbem_destroy(c); return STBEM_EHIP; }
    }
    if ((rc = build_block_lists(c))) { stbem_destroy(c); return rc; }
    c->m0ord.qs_near = 12; c->m0ord.qt_near = 12; c->m0ord.near_ratio = 0.5;
    c->m0ord.q_tol = c->ord.q_tol; c->m0ord.z_floor = c->ord.z_floor;
    c->m0ord.omax = 0.0;
    for (int t = 0; t < c->ntri; ++t)
        for (int e = 0; e < 3; ++e) {
            int a = c->tri[3 * t + e], b = c->tri[3 * t + (e + 1) % 3];
            double d = std::hypot(c->ox[a] - c->ox[b], c->oy[a] - c->oy[b]);
            if (d > c->m0ord.omax) c->m0ord.omax = d;
        }
    {
        // M0 rows k >= 1: power series of ln(t1/t0) + Ein(a/t1) - Ein(a/t0) in
        // a = alpha r^2 / 4, used for pairs with a/t0 <= 4 (the alternating
        // terms reach at most 4^4/4! = 10.7 times the leading one while the sum
        // is >= e^{-4} of it: < 1e-13 relative rounding); R = the diameter of
        // the bounding box of Gamma_h and Omega_h bounds r
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
        for (int v = 0; v < c->ng; ++v) { xmin = std::fmin(xmin, c->vx[v]); xmax = std::fmax(xmax, c->vx[v]); ymin = std::fmin(ymin, c->vy[v]); ymax = std::fmax(ymax, c->vy[v]); }
        for (int v = 0; v < c->nv; ++v) { xmin = std::fmin(xmin, c->ox[v]); xmax = std::fmax(xmax, c->ox[v]); ymin = std::fmin(ymin, c->oy[v]); ymax = std::fmax(ymax, c->oy[v]); }
        double R2 = (xmax - xmin) * (xmax - xmin) + (ymax - ymin) * (ymax - ymin);
        double amax = 0.25 * c->alpha * R2;
        std::vector<double> cf((size_t)c->nt * kPolyMax, 0.0), cfd((size_t)c->nt * kPolyMax, 0.0);
        std::vector<int> nn(c->nt, 0);
        std::vector<double> am(c->nt, 0.0), it(c->nt + 1, 0.0), es(c->nt, 0.0);
        std::vector<double> ce((size_t)c->nt * kEconMax, 0.0), cde((size_t)c->nt * kEconMax, 0.0);
        for (int k = 1; k <= c->nt; ++k) it[k] = 1.0 / c->t[k];
        for (int k = 1; k < c->nt; ++k) {
            long double t0 = c->t[k], t1 = c->t[k + 1], h = (long double)c->t[k + 1] - (long double)c->t[k];
            double amk = std::fmin(4.0 * c->t[k], amax);   // the series is used for a <= amk
            am[k] = amk;
            double* co = &cf[(size_t)k * kPolyMax];
            double* cd = &cfd[(size_t)k * kPolyMax];
            long double cl[kPolyMax], cdl[kPolyMax];
            cl[0] = cdl[0] = logl(t1 / t0);
            co[0] = cd[0] = (double)cl[0];
            long double fact = 1, sum = 0, pw1 = 1, pw0 = 1;   // sum = sum_j t1^j t0^(n-1-j)
            int n = 1;
            bool conv = false;
            for (; n < kPolyMax; ++n) {
                // t1^-n - t0^-n = -h * S_n / (t0 t1)^n,  S_n = sum_{j<n} t1^j t0^{n-1-j}
                sum = sum * t0 + pw1;           // S_n = t0 S_{n-1} + t1^{n-1}
                pw1 *= t1; pw0 *= t0;
                fact *= n;
                long double en = -h * sum / (pw1 * pw0) / fact;  // (t1^-n - t0^-n)/n!
                long double sg = (n & 1) ? 1.0L : -1.0L;       // (-1)^{n+1}
                cl[n] = sg * en / n;
                cdl[n] = sg * en * (1.0L / n + 1.0L);
                co[n] = (double)cl[n];
                cd[n] = (double)cdl[n];
                long double tail = powl(amk / t0, n) / fact;
                if (tail < 1e-18L * fabsl((long double)co[0]) && n > 2) { ++n; conv = true; break; }
            }
            nn[k] = conv ? n : 0;      // not converged: the E1 path is used
            if (nn[k] > 0) {
                es[k] = (double)(2.0L / amk);
                if (!econ_poly(cl, n, amk, 1e-18L, &ce[(size_t)k * kEconMax]) ||
                    !econ_poly(cdl, n, amk, 1e-18L, &cde[(size_t)k * kEconMax]))
                    nn[k] = 0;
            }
        }
        // rows whose series covers every pair (amax reached) from ksplit on
        c->m0_ksplit = c->nt;
        c->m0_npow = 0;
        for (int k = c->nt - 1; k >= 1 && nn[k] > 0 && am[k] >= amax; --k) c->m0_ksplit = k;
        for (int k = c->m0_ksplit; k < c->nt; ++k) c->m0_npow = std::max(c->m0_npow, nn[k]);
        int rc2 = 0;
        if ((rc2 = upload(c, &c->d_m0c, cf)) || (rc2 = upload(c, &c->d_m0cd, cfd)) || (rc2 = upload(c, &c->d_m0n, nn)) ||
            (rc2 = upload(c, &c->d_m0amax, am)) || (rc2 = upload(c, &c->d_m0it, it)) ||
            (rc2 = upload(c, &c->d_m0ce, ce)) || (rc2 = upload(c, &c->d_m0cde, cde)) || (rc2 = upload(c, &c->d_m0es, es))) {
            stbem_destroy(c);
            return rc2;
        }
    }
    *out = c;
    return STBEM_OK;
}

int stbem_destroy(stbem_ctx* c)
{
    if (!c) return STBEM_OK;
    for (int s = 0; s < 7; ++s) dev_free(c, c->mat[s]);
    free_f32(c, true, true);
    void* own[] = {c->d_t, c->d_vx, c->d_vy, c->d_ex, c->d_ey, c->d_len, c->d_ox, c->d_oy, c->d_mt, c->d_m0c, c->d_m0cd, c->d_m0n, c->d_m0amax, c->d_m0it, c->d_m0ce, c->d_m0cde, c->d_m0es, c->d_v2t_loc,
                   c->d_tri, c->d_v2t_ptr, c->d_v2t, c->d_tab, c->d_m0tab, c->part, c->d_tbs, c->d_tbs32, c->wvec,
                   c->gm_q, c->gm_part, c->gm_h, c->gm_v};
    for (void* p : own) if (p) (void)hipFree(p);
    for (int q = 0; q < 7; ++q) if (c->d_blist[q]) (void)hipFree(c->d_blist[q]);
    if (c->d_klist_fused) (void)hipFree(c->d_klist_fused);
    clear_timing(c);
    delete c;
    return STBEM_OK;
}

int stbem_set_toeplitz(stbem_ctx* c, int on)
{
    if (!c) return STBEM_EINVAL;
    const bool want = on != 0;
    if (want) {
        const double h0 = c->t[1] - c->t[0];
        for (int k = 1; k < c->nt; ++k)
            if (std::fabs((c->t[k + 1] - c->t[k]) - h0) > 1e-12 * h0)
                return fail(c, STBEM_EINVAL, "block-Toeplitz storage needs uniform time steps (step %d differs)", k);
    }
    if (want == c->toep) return STBEM_OK;
    // the storage format changes: drop the causal operators and FP32 copies
    (void)hipDeviceSynchronize();
    const int slots[5] = {0, 1, 2, 4, 5};
    for (int e = 0; e < 5; ++e) free_slot(c, slots[e]);
    free_f32(c, true, true);
    c->toep = want;
    for (int q = 0; q < 7; ++q) if (c->d_blist[q]) { (void)hipFree(c->d_blist[q]); c->d_blist[q] = nullptr; }
    if (c->d_klist_fused) { (void)hipFree(c->d_klist_fused); c->d_klist_fused = nullptr; }
    return build_block_lists(c);
}

int stbem_potential(stbem_ctx* c, long long npts, const double* pts, const double* w, const double* gd,
                    const double* u0, double* out, void* stream)
{
    if (!c || npts < 0 || (npts > 0 && (!pts || !w || !gd || !out))) return STBEM_EINVAL;
    if (u0 && c->nv == 0) return fail(c, STBEM_EINVAL, "u0 given but no Omega mesh");
    if (npts == 0) return STBEM_OK;
    if (npts > 0x7fffffffLL) return fail(c, STBEM_EINVAL, "too many points");
    hipStream_t s = S(stream);
    // validate on the host: 0 < t <= T and x strictly inside the polygon
    std::vector<double> hp((size_t)npts * 3);
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(hp.data(), pts, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
    double lmin = 1e300;
    for (int i = 0; i < c->ng; ++i) lmin = std::fmin(lmin, c->len[i]);
    for (long long e = 0; e < npts; ++e) {
        const double x = hp[3 * e], y = hp[3 * e + 1], t = hp[3 * e + 2];
        if (!(t > 0.0) || !(t <= c->t[c->nt])) return fail(c, STBEM_EINVAL, "point %lld: t = %g outside (0, T]", e, t);
        bool in = false;
        double dmin = 1e300;
        for (int i = 0; i < c->ng; ++i) {
            const int j = i + 1 == c->ng ? 0 : i + 1;
            const double ax = c->vx[i], ay = c->vy[i], bx = c->vx[j], by = c->vy[j];
            if ((ay > y) != (by > y) && x < ax + (y - ay) * (bx - ax) / (by - ay)) in = !in;
            double u = ((x - ax) * c->ex[i] + (y - ay) * c->ey[i]) / c->len[i];
            u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
            dmin = std::fmin(dmin, std::hypot(x - ax - u * (bx - ax), y - ay - u * (by - ay)));
        }
        if (!in || dmin <= 1e-12 * lmin) return fail(c, STBEM_EINVAL, "point %lld is not inside Omega", e);
    }
    {
        KTimer kt(c, "k_pot_bnd", (double)npts, s);
        hipLaunchKernelGGL(k_pot_bnd, dim3((unsigned)npts), dim3(kWG), 0, s, geom(c), c->d_tab, c->ord, pts, w, gd,
                           u0 ? 1 : 0, out);
    }
    if (u0) {
        KTimer kt(c, "k_pot_init", (double)npts, s);
        hipLaunchKernelGGL(k_pot_init, dim3((unsigned)npts), dim3(kWG), 0, s, geom(c), mesh(c), c->d_tab, c->ord, pts, u0, out);
    }
    HIPCHK(c, hipGetLastError());
    return STBEM_OK;
}

int stbem_set_timing(stbem_ctx* c, int on)
{
    if (!c) return STBEM_EINVAL;
    for (auto& r : c->trecs) (void)hipEventSynchronize(r.b);
    clear_timing(c);
    c->timing = on != 0;
    return STBEM_OK;
}

int stbem_kernel_times(stbem_ctx* c, stbem_kernel_time* out, int cap)
{
    if (!c || (cap > 0 && !out) || cap < 0) return STBEM_EINVAL;
    std::vector<stbem_kernel_time> agg;
    for (auto& r : c->trecs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(c, STBEM_EHIP, "timing event");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(c, STBEM_EHIP, "timing event");
        size_t e = 0;
        while (e < agg.size() && r.name != agg[e].name) ++e;
        if (e == agg.size()) {
            stbem_kernel_time k;
            memset(&k, 0, sizeof k);
            snprintf(k.name, sizeof k.name, "%s", r.name.c_str());
            agg.push_back(k);
        }
        agg[e].launches += 1;
        agg[e].ms += ms;
        agg[e].units += r.units;
        agg[e].flops += r.flops;
    }
    for (size_t e = 0; e < agg.size() && (int)e < cap; ++e) out[e] = agg[e];
    return (int)agg.size();
}

int stbem_set_allocator(stbem_ctx* c, stbem_alloc_fn alloc, stbem_free_fn release, void* user)
{
    if (!c || (!alloc) != (!release)) return STBEM_EINVAL;
    for (int s = 0; s < 7; ++s)
        if (c->mat[s]) return fail(c, STBEM_EINVAL, "set the allocator before assembling");
    c->alloc = alloc; c->release = release; c->user = user;
    return STBEM_OK;
}

int stbem_sizes(const stbem_ctx* c, long long* n, int* ng, int* nt, int* nv, long long* packed)
{
    if (!c) return STBEM_EINVAL;
    if (n) *n = c->n;
    if (ng) *ng = c->ng;
    if (nt) *nt = c->nt;
    if (nv) *nv = c->nv;
    if (packed) *packed = c->packed;
    return STBEM_OK;
}

int stbem_assemble(stbem_ctx* c, unsigned mask, int precision, void* stream)
{
    if (!c) return STBEM_EINVAL;
    if (mask == 0 || (mask & ~127u)) return fail(c, STBEM_EINVAL, "bad operator mask %u", mask);
    if (precision != STBEM_FP64 && precision != STBEM_FP32_IR) return fail(c, STBEM_EINVAL, "unknown precision %d", precision);
    if (precision == STBEM_FP32_IR) {
        if (mask & ~(STBEM_V | STBEM_D)) return fail(c, STBEM_EINVAL, "FP32 storage is for V_h and D_h only");
        if (c->toep) return fail(c, STBEM_EINVAL, "FP32 storage needs packed storage (block-Toeplitz mode is FP64 only)");
    }
    const unsigned ops[7] = {STBEM_V, STBEM_K, STBEM_D, STBEM_M0, STBEM_DV, STBEM_DK, STBEM_DM0};
    // V_h and D_h together: V_h's separated blocks are computed by D_h's far
    // tiles (same block lists); V is assembled first, so its storage exists
    const bool fuse = (mask & STBEM_V) && (mask & STBEM_D) && c->vd_fusable;
    // K_h too (FP64): its separated blocks from the same tiles; K is
    // assembled before D, so its storage exists when D's far tiles run
    const bool fuse_k = fuse && (mask & STBEM_K) && precision == STBEM_FP64;
    for (unsigned op : ops)
        if (mask & op) {
            int rc = assemble_one(c, op, S(stream), fuse, precision, fuse_k);
            if (rc) return rc;
        }
    return STBEM_OK;
}

int stbem_release(stbem_ctx* c, unsigned mask)
{
    if (!c) return STBEM_EINVAL;
    if (mask & ~127u) return fail(c, STBEM_EINVAL, "bad operator mask %u", mask);
    const unsigned ops[7] = {STBEM_V, STBEM_K, STBEM_D, STBEM_M0, STBEM_DV, STBEM_DK, STBEM_DM0};
    for (unsigned op : ops)
        if (mask & op) {
            free_slot(c, op_slot(op));
            if (op == STBEM_V || op == STBEM_D) free_f32(c, op == STBEM_V, op == STBEM_D);
        }
    return STBEM_OK;
}

int stbem_matrix(stbem_ctx* c, unsigned op, const double** ptr, size_t* bytes)
{
    if (!c || !ptr) return STBEM_EINVAL;
    int slot = op_slot(op);
    if (slot < 0) return fail(c, STBEM_EINVAL, "unknown operator %u", op);
    if (!c->mat[slot]) return fail(c, STBEM_ENOTASSEMBLED, "operator %u not assembled", op);
    *ptr = c->mat[slot];
    if (bytes) *bytes = c->mat_bytes[slot];
    return STBEM_OK;
}

int stbem_matrix_f32(stbem_ctx* c, unsigned op, const float** hi, const float** lo, size_t* bytes)
{
    if (!c || !hi) return STBEM_EINVAL;
    if (op != STBEM_V && op != STBEM_D) return fail(c, STBEM_EINVAL, "FP32 storage exists for V_h and D_h only");
    const float* h = op == STBEM_V ? c->v_hi : c->d_32;
    if (!h) return fail(c, STBEM_ENOTASSEMBLED, "operator %u has no FP32 storage", op);
    *hi = h;
    if (lo) *lo = op == STBEM_V ? c->v_lo : nullptr;
    if (bytes) *bytes = (size_t)causal_entries(c) * sizeof(float);
    return STBEM_OK;
}

int stbem_apply(stbem_ctx* c, unsigned op, int trans, const double* x, double* y, void* stream)
{
    if (!c || !x || !y) return STBEM_EINVAL;
    int slot = op_slot(op);
    if (slot < 0) return fail(c, STBEM_EINVAL, "unknown operator %u", op);
    if (!c->mat[slot]) {
        // V_h or D_h held in FP32 storage only
        if (op == STBEM_V && c->v_hi && c->v_lo) return packed_apply(c, nullptr, c->v_hi, c->v_lo, nullptr, trans ? 1 : 0, x, y, S(stream));
        if (op == STBEM_D && c->d_32) return packed_apply(c, nullptr, nullptr, nullptr, c->d_32, trans ? 1 : 0, x, y, S(stream));
        return fail(c, STBEM_ENOTASSEMBLED, "operator %u not assembled", op);
    }
    if (op == STBEM_M0 || op == STBEM_DM0) return dense_apply(c, c->mat[slot], trans ? 1 : 0, x, y, S(stream));
    return packed_apply(c, c->mat[slot], nullptr, nullptr, nullptr, trans ? 1 : 0, x, y, S(stream));
}

int stbem_apply_noalloc(stbem_ctx* c, unsigned op, int trans, const double* x, double* y, void* stream)
{
    if (!c || !x || !y) return STBEM_EINVAL;
    if (op == STBEM_M0 || op == STBEM_DM0) return fail(c, STBEM_EINVAL, "stbem_apply_noalloc: causal operators only");
    int slot = op_slot(op);
    if (slot < 0) return fail(c, STBEM_EINVAL, "unknown operator %u", op);
    if (c->toep) return fail(c, STBEM_EINVAL, "stbem_apply_noalloc: packed storage only (not block-Toeplitz mode)");
    if (!c->noalloc) return fail(c, STBEM_EHIP, "stbem_apply_noalloc: no scratch address for this context");
    const double* A = c->mat[slot];
    const float *hi = nullptr, *lo = nullptr, *a32 = nullptr;
    if (!A) {
        if (op == STBEM_V && c->v_hi && c->v_lo) { hi = c->v_hi; lo = c->v_lo; }
        else if (op == STBEM_D && c->d_32) a32 = c->d_32;
        else return fail(c, STBEM_ENOTASSEMBLED, "operator %u not assembled", op);
    }
    const long long ng = c->ng;
    if ((long long)c->nt * ng > kNoAllocDoubles)
        return fail(c, STBEM_EINVAL, "stbem_apply_noalloc: one block row needs %lld partials, the scratch holds %lld",
                    (long long)c->nt * ng, kNoAllocDoubles);
    hipStream_t s = S(stream);
    int k0 = 0;
    while (k0 < c->nt) {
        // the most block rows whose partials fit the scratch
        int k1 = k0 + 1;
        const long long pb0 = (long long)k0 * (k0 + 1) / 2;
        while (k1 < c->nt && ((long long)(k1 + 1) * (k1 + 2) / 2 - pb0) * ng <= kNoAllocDoubles) ++k1;
        const long long nb = (long long)k1 * (k1 + 1) / 2 - pb0;
        int rc = gemv_partials(c, A, hi, lo, a32, trans ? 1 : 0, x, c->noalloc, pb0, nb, s);
        if (!rc) rc = gemv_reduce(c, c->noalloc, y, trans ? 1 : 0, k0, k1, s);
        if (rc) return rc;
        k0 = k1;
    }
    return STBEM_OK;
}

int stbem_mass(stbem_ctx* c, int trans, const double* x, double* y, void* stream)
{
    if (!c || !x || !y) return STBEM_EINVAL;
    hipLaunchKernelGGL(k_mass, dim3(grid1(c->n)), dim3(kWG), 0, S(stream), c->d_t, c->d_len, x, y, c->ng, c->nt,
                       trans ? 1 : 0, 1.0, (const double*)nullptr);
    HIPCHK(c, hipGetLastError());
    return STBEM_OK;
}

// z = Mt^-1 D_h Mt^-1 r (D_h^T for trans), D_h from d32 if given, else the
// stored D_h (FP64, or FP32 when D_h was assembled in FP32_IR); tmp: N doubles
static int precondition_impl(stbem_ctx* c, int trans, const double* r, double* z, double* tmp, const float* d32,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_div, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, r, (const double*)c->d_mt, tmp);
    HIPCHK(c, hipGetLastError());
    if (!d32 && !c->mat[2]) d32 = c->d_32;
    int rc = d32 ? packed_apply(c, nullptr, nullptr, nullptr, d32, trans, tmp, z, s)
                 : packed_apply(c, c->mat[2], nullptr, nullptr, nullptr, trans, tmp, z, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_div, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, (const double*)z, (const double*)c->d_mt, z);
    HIPCHK(c, hipGetLastError());
    return 0;
}

int stbem_precondition(stbem_ctx* c, int trans, const double* r, double* z, void* stream)
{
    if (!c || !r || !z) return STBEM_EINVAL;
    if (!c->mat[2] && !c->d_32) return fail(c, STBEM_ENOTASSEMBLED, "D_h not assembled");
    int rc = ensure_wvec(c, 2);
    if (rc) return rc;
    return precondition_impl(c, trans ? 1 : 0, r, z, c->wvec, nullptr, S(stream));
}

int stbem_rhs(stbem_ctx* c, const double* g, const double* u0, double* f, void* stream)
{
    if (!c || !g || !f) return STBEM_EINVAL;
    if (!c->mat[1]) return fail(c, STBEM_ENOTASSEMBLED, "K_h not assembled");
    if (u0 && !c->mat[3] && c->nv == 0) return fail(c, STBEM_EINVAL, "u0 given but no Omega mesh");
    hipStream_t s = S(stream);
    int rc = ensure_wvec(c, 2);
    if (rc) return rc;
    double* tmp = c->wvec;
    // tmp = K g;  f = 1/2 M g + tmp;  f -= M0 u0
    if ((rc = packed_apply(c, c->mat[1], nullptr, nullptr, nullptr, 0, g, tmp, s))) return rc;
    hipLaunchKernelGGL(k_mass, dim3(grid1(c->n)), dim3(kWG), 0, s, c->d_t, c->d_len, g, f, c->ng, c->nt, 0, 0.5,
                       (const double*)tmp);
    HIPCHK(c, hipGetLastError());
    if (u0) {
        // M0 u0 from the stored matrix, or computed row chunk by row chunk
        if ((rc = c->mat[3] ? dense_apply(c, c->mat[3], 0, u0, tmp, s) : m0_fused_apply(c, u0, tmp, s))) return rc;
        hipLaunchKernelGGL(k_axpby, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, -1.0, (const double*)tmp, 1.0, f);
        HIPCHK(c, hipGetLastError());
    }
    return STBEM_OK;
}

int stbem_rhs_adjoint(stbem_ctx* c, const double* lam, double* out, void* stream)
{
    if (!c || !lam || !out) return STBEM_EINVAL;
    if (!c->mat[1]) return fail(c, STBEM_ENOTASSEMBLED, "K_h not assembled");
    hipStream_t s = S(stream);
    int rc = ensure_wvec(c, 2);
    if (rc) return rc;
    double* tmp = c->wvec;
    // tmp = K^T lam;  out = 1/2 M^T lam + tmp
    if ((rc = packed_apply(c, c->mat[1], nullptr, nullptr, nullptr, 1, lam, tmp, s))) return rc;
    hipLaunchKernelGGL(k_mass, dim3(grid1(c->n)), dim3(kWG), 0, s, c->d_t, c->d_len, lam, out, c->ng, c->nt, 1, 0.5,
                       (const double*)tmp);
    HIPCHK(c, hipGetLastError());
    return STBEM_OK;
}

// ----------------------------------------------------------------- GMRES
namespace {

struct SolveOp {
    stbem_ctx* c;
    int trans, precond;
    const double* A; const float *hi, *lo, *a32;     // system matrix storage
    const float* d32;                                // FP32 D (else FP64 D)
    double* tmp;
};

int op_apply(const SolveOp& o, const double* x, double* y, hipStream_t s)
{
    // y = C A x   (C = Mt^-1 D Mt^-1 or identity)
    stbem_ctx* c = o.c;
    if (!o.precond) return packed_apply(c, o.A, o.hi, o.lo, o.a32, o.trans, x, y, s);
    int rc = packed_apply(c, o.A, o.hi, o.lo, o.a32, o.trans, x, o.tmp + c->n, s);
    if (rc) return rc;
    return precondition_impl(c, o.trans, o.tmp + c->n, y, o.tmp, o.d32, s);
}

int op_precond(const SolveOp& o, const double* r, double* z, hipStream_t s)
{
    stbem_ctx* c = o.c;
    if (!o.precond) {
        HIPCHK(c, hipMemcpyAsync(z, r, (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        return 0;
    }
    return precondition_impl(c, o.trans, r, z, o.tmp, o.d32, s);
}

// GMRES workspace for up to maxit iterations, kept by the context
int ensure_gmres(stbem_ctx* c, int maxit)
{
    if (c->gm_q && c->gm_cap >= maxit) return 0;
    double* own[4] = {c->gm_q, c->gm_part, c->gm_h, c->gm_v};
    for (double* p : own) if (p) (void)hipFree(p);
    c->gm_q = c->gm_part = c->gm_h = c->gm_v = nullptr;
    c->gm_cap = 0;
    const long long n = c->n, nchunk = (n + kDotChunk - 1) / kDotChunk;
    if (hipMalloc((void**)&c->gm_q, (size_t)(maxit + 1) * n * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->gm_part, (size_t)(maxit + 1) * nchunk * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->gm_h, (size_t)(maxit + 2) * 2 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->gm_v, (size_t)n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        double* got[4] = {c->gm_q, c->gm_part, c->gm_h, c->gm_v};
        for (double* p : got) if (p) (void)hipFree(p);
        c->gm_q = c->gm_part = c->gm_h = c->gm_v = nullptr;
        return fail(c, STBEM_ENOMEM, "GMRES workspace (%d vectors of %lld)", maxit + 1, n);
    }
    c->gm_cap = maxit;
    return 0;
}

// left-preconditioned GMRES, x0 = 0, CGS2 orthogonalisation in FP64
int gmres(const SolveOp& o, const double* f, double* w, double tol, int maxit, int* iters, double* relres, hipStream_t s)
{
    stbem_ctx* c = o.c;
    const long long n = c->n;
    const long long ldq = n;
    if (int rcw = ensure_gmres(c, maxit)) return rcw;
    double* Q = c->gm_q;
    DotWork dw;
    dw.nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
    dw.part = c->gm_part;
    double* hdev = c->gm_h;
    double* v = c->gm_v;
    std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), gv(maxit + 1, 0.0), hh(2 * (maxit + 2));
    int rc = 0, j = 0;
    double beta = 0.0;
    *iters = 0; *relres = 0.0;
    // r0 = C f
    if ((rc = op_precond(o, f, Q, s))) goto out;
    if ((rc = dots(c, dw, Q, ldq, 1, Q, hdev, s))) goto out;
    HIPCHK(c, hipMemcpyAsync(hh.data(), hdev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    beta = std::sqrt(hh[0]);
    if (beta == 0.0) {
        hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(kWG), 0, s, n, 0.0, w);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(s));
        goto out;
    }
    hipLaunchKernelGGL(k_axpby, dim3(grid1(n)), dim3(kWG), 0, s, n, 1.0 / beta, (const double*)Q, 0.0, Q);
    gv[0] = beta;
    for (j = 0; j < maxit; ++j) {
        double* qj1 = Q + (long long)(j + 1) * ldq;
        if ((rc = op_apply(o, Q + (long long)j * ldq, v, s))) goto out;
        // classical Gram-Schmidt, twice: the coefficients stay on the device
        // for the subtraction (pass p at hdev + p (maxit + 1), the norm after
        // them), so the host waits once per iteration
        for (int pass = 0; pass < 2; ++pass) {
            double* hp = hdev + (size_t)pass * (maxit + 1);
            if ((rc = dots(c, dw, Q, ldq, j + 1, v, hp, s))) goto out;
            hipLaunchKernelGGL(k_basis_sub, dim3(grid1(n)), dim3(kWG), 0, s, (const double*)Q, ldq, j + 1, (const double*)hp, v, n);
        }
        if ((rc = dots(c, dw, v, ldq, 1, v, hdev + (size_t)2 * (maxit + 1), s))) goto out;
        HIPCHK(c, hipMemcpyAsync(hh.data(), hdev, (size_t)(2 * (maxit + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i <= j; ++i) H[(size_t)j * (maxit + 1) + i] += hh[(size_t)pass * (maxit + 1) + i];
        {
            double hn = std::sqrt(hh[(size_t)2 * (maxit + 1)]);
            double* col = &H[(size_t)j * (maxit + 1)];
            col[j + 1] = hn;
            if (hn > 0.0)
                hipLaunchKernelGGL(k_axpby, dim3(grid1(n)), dim3(kWG), 0, s, n, 1.0 / hn, (const double*)v, 0.0, qj1);
            for (int i = 0; i < j; ++i) {
                double a = col[i], b = col[i + 1];
                col[i] = cs[i] * a + sn[i] * b;
                col[i + 1] = -sn[i] * a + cs[i] * b;
            }
            double a = col[j], b = col[j + 1], r = std::hypot(a, b);
            cs[j] = a / r; sn[j] = b / r;
            col[j] = r; col[j + 1] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            *relres = std::fabs(gv[j + 1]) / beta;
            if (std::fabs(gv[j + 1]) <= tol * beta || hn == 0.0) { ++j; break; }
        }
    }
    if (j > maxit) j = maxit;
    {
        // back substitution on the host, combination on the device
        std::vector<double> y(j);
        for (int i = j - 1; i >= 0; --i) {
            double sacc = gv[i];
            for (int l = i + 1; l < j; ++l) sacc -= H[(size_t)l * (maxit + 1) + i] * y[l];
            y[i] = sacc / H[(size_t)i * (maxit + 1) + i];
        }
        HIPCHK(c, hipMemcpyAsync(hdev, y.data(), (size_t)j * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_basis_comb, dim3(grid1(n)), dim3(kWG), 0, s, (const double*)Q, ldq, j, (const double*)hdev, w, n, 0);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(s));
    }
    *iters = j;
out:
    return rc;
}

int true_relres(stbem_ctx* c, const SolveOp& o64, const double* f, const double* w, double* r, double* res, hipStream_t s)
{
    // r = f - A w in FP64 storage (or hi+lo), returns ||r|| / ||f||
    int rc = packed_apply(c, o64.A, o64.hi, o64.lo, nullptr, o64.trans, w, r, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, 1.0, f, -1.0, r);
    if ((rc = ensure_gmres(c, 1))) return rc;
    DotWork dw;
    dw.nchunk = (int)((c->n + kDotChunk - 1) / kDotChunk);
    dw.part = c->gm_part;
    double* hd = c->gm_h;
    double hh[2];
    if ((rc = dots(c, dw, r, c->n, 1, r, hd, s)) || (rc = dots(c, dw, f, c->n, 1, f, hd + 1, s))) return rc;
    HIPCHK(c, hipMemcpyAsync(hh, hd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *res = hh[1] > 0 ? std::sqrt(hh[0] / hh[1]) : 0.0;
    return 0;
}

}  // namespace

int stbem_prepare_ir(stbem_ctx* c, void* stream)
{
    if (!c) return STBEM_EINVAL;
    if (c->toep) return fail(c, STBEM_EINVAL, "FP32 refinement needs packed storage (block-Toeplitz mode is FP64 only)");
    if (!c->mat[0] && !c->v_hi) return fail(c, STBEM_ENOTASSEMBLED, "V_h not assembled");
    hipStream_t s = S(stream);
    const size_t fb = (size_t)c->packed * sizeof(float);
    const unsigned gs = (unsigned)std::min<long long>(grid1(c->packed), 1LL << 20);   // grid-stride
    // FP64 V_h resident: the inner solves read hi = fl32(V), the outer
    // residual reads the FP64 V_h itself (no lo part is kept)
    if (c->mat[0] && !c->v_hi) {
        c->v_hi = (float*)dev_alloc(c, fb);
        if (!c->v_hi) return fail(c, STBEM_ENOMEM, "FP32 copy of V_h (%zu bytes)", fb);
        hipLaunchKernelGGL(k_split, dim3(gs), dim3(kWG), 0, s, c->packed, (const double*)c->mat[0], c->v_hi, (float*)nullptr);
    }
    if (c->mat[2] && !c->d_32) {
        c->d_32 = (float*)dev_alloc(c, fb);
        if (!c->d_32) return fail(c, STBEM_ENOMEM, "FP32 copy of D_h (%zu bytes)", fb);
        hipLaunchKernelGGL(k_split, dim3(gs), dim3(kWG), 0, s, c->packed, (const double*)c->mat[2], c->d_32, (float*)nullptr);
    }
    HIPCHK(c, hipGetLastError());
    return STBEM_OK;
}

int stbem_solve(stbem_ctx* c, const double* f, double* w, const stbem_solve_opts* opts, stbem_solve_info* info, void* stream)
{
    if (!c || !f || !w || !opts) return STBEM_EINVAL;
    if (opts->max_it < 1 || !(opts->tol > 0)) return fail(c, STBEM_EINVAL, "bad tolerance or iteration limit");
    if (opts->mode != STBEM_FP64 && opts->mode != STBEM_FP32_IR) return fail(c, STBEM_EINVAL, "unknown solve mode %d", opts->mode);
    const bool ir = opts->mode == STBEM_FP32_IR;
    if (!c->mat[0] && !(ir && c->v_hi)) {
        if (c->v_hi) return fail(c, STBEM_ENOTASSEMBLED, "V_h is held in FP32 storage only: use the FP32_IR mode");
        return fail(c, STBEM_ENOTASSEMBLED, "V_h not assembled");
    }
    if (opts->precondition && !c->mat[2] && !(ir && c->d_32)) return fail(c, STBEM_ENOTASSEMBLED, "D_h not assembled");
    hipStream_t s = S(stream);
    stbem_solve_info inf = {0, 0, 0.0, 0.0};
    int rc = ensure_wvec(c, 5);
    if (rc) return rc;
    double* tmp = c->wvec;                       // 3 vectors for the operators; r and the correction
    SolveOp o64 = {c, opts->trans ? 1 : 0, opts->precondition ? 1 : 0, c->mat[0], nullptr, nullptr, nullptr, nullptr, tmp};
    if (!ir) {
        int it = 0;
        double rr = 0.0;
        rc = gmres(o64, f, w, opts->tol, opts->max_it, &it, &rr, s);
        inf.iters = it; inf.relres = rr;
        if (!rc) rc = true_relres(c, o64, f, w, tmp + 2 * c->n, &inf.true_relres, s);
        if (!rc && rr > opts->tol) rc = STBEM_WARN_NOT_CONVERGED;
    } else {
        if (!c->v_hi || (opts->precondition && !c->d_32 && c->mat[2])) {
            if ((rc = stbem_prepare_ir(c, stream))) return rc;
        }
        // outer: r = f - V w in FP64 (the FP64 V_h when resident, else the
        // pair hi + lo, accurate to about 2^-48); inner: GMRES on FP32 V_hi
        // with the FP32 D_h in the preconditioner; w += correction
        SolveOp ores = c->mat[0] ? o64 : SolveOp{c, o64.trans, 0, nullptr, c->v_hi, c->v_lo, nullptr, nullptr, tmp};
        SolveOp o32 = {c, o64.trans, opts->precondition ? 1 : 0, nullptr, nullptr, nullptr, c->v_hi, c->d_32, tmp};
        double* r = tmp + 3 * c->n;
        double* corr = tmp + 4 * c->n;
        hipLaunchKernelGGL(k_fill, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, 0.0, w);
        HIPCHK(c, hipGetLastError());
        double prev = 1e300, res = 0.0;
        int outer = 0;
        for (;;) {
            if ((rc = true_relres(c, ores, f, w, r, &res, s))) break;
            if (res <= opts->ir_tol) break;
            if (outer >= opts->max_outer) { rc = STBEM_WARN_NOT_CONVERGED; break; }
            if (res > 0.5 * prev) { rc = STBEM_WARN_IR_STAGNATION; break; }
            prev = res;
            int it = 0;
            double rr = 0.0;
            if ((rc = gmres(o32, r, corr, opts->inner_tol, opts->max_it, &it, &rr, s))) break;
            inf.iters += it;
            inf.relres = rr;
            hipLaunchKernelGGL(k_axpby, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, 1.0, (const double*)corr, 1.0, w);
            ++outer;
        }
        inf.outer = outer;
        inf.true_relres = res;
        if (rc == 0 || rc == STBEM_WARN_NOT_CONVERGED || rc == STBEM_WARN_IR_STAGNATION) {
            int rc2 = true_relres(c, ores, f, w, r, &inf.true_relres, s);
            if (rc2) rc = rc2;
        }
    }
    (void)hipStreamSynchronize(s);
    if (info) *info = inf;
    return rc;
}

int stbem_grad_alpha(stbem_ctx* c, const double* lam, const double* w, const double* g, const double* u0,
                     double* out, void* stream)
{
    if (!c || !lam || !w || !g || !out) return STBEM_EINVAL;
    if (u0 && c->nv == 0) return fail(c, STBEM_EINVAL, "u0 given but no Omega mesh");
    hipStream_t s = S(stream);
    int rc = ensure_wvec(c, 2);
    if (rc || (rc = ensure_gmres(c, 1))) return rc;
    double* t = c->wvec;
    // t = dK g - dV w - dM0 u0, each product from the stored matrix or, when
    // it is not assembled, recomputed block row range by range
    rc = c->mat[5] ? packed_apply(c, c->mat[5], nullptr, nullptr, nullptr, 0, g, t, s) : deriv_apply_blockwise(c, 5, g, t, s);
    if (rc) return rc;
    rc = c->mat[4] ? packed_apply(c, c->mat[4], nullptr, nullptr, nullptr, 0, w, t + c->n, s)
                   : deriv_apply_blockwise(c, 4, w, t + c->n, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, -1.0, (const double*)(t + c->n), 1.0, t);
    if (u0) {
        rc = c->mat[6] ? dense_apply(c, c->mat[6], 0, u0, t + c->n, s) : m0_fused_apply(c, u0, t + c->n, s, true);
        if (rc) return rc;
        hipLaunchKernelGGL(k_axpby, dim3(grid1(c->n)), dim3(kWG), 0, s, c->n, -1.0, (const double*)(t + c->n), 1.0, t);
    }
    DotWork dw;
    dw.nchunk = (int)((c->n + kDotChunk - 1) / kDotChunk);
    dw.part = c->gm_part;
    return dots(c, dw, lam, c->n, 1, t, out, s);
}

int stbem_entries(stbem_ctx* c, unsigned op, long long n, const int* idx, double* out, void* stream)
{
    if (!c || (n > 0 && (!idx || !out))) return STBEM_EINVAL;
    if (n == 0) return STBEM_OK;
    if (n > kMaxWG * kWG) return fail(c, STBEM_EINVAL, "at most %lld entries per call", kMaxWG * kWG);
    hipStream_t s = S(stream);
    unsigned nwg = (unsigned)grid1(n);
    Geom g = geom(c);
    switch (op) {
    case STBEM_V: hipLaunchKernelGGL(k_entries<OP_V>, dim3(nwg), dim3(kWG), 0, s, g, c->d_tab, c->ord, c->lmax, n, idx, out); break;
    case STBEM_K: hipLaunchKernelGGL(k_entries<OP_K>, dim3(nwg), dim3(kWG), 0, s, g, c->d_tab, c->ord, c->lmax, n, idx, out); break;
    case STBEM_D: hipLaunchKernelGGL(k_entries<OP_D>, dim3(nwg), dim3(kWG), 0, s, g, c->d_tab, c->ord, c->lmax, n, idx, out); break;
    case STBEM_DV: hipLaunchKernelGGL(k_entries<OP_DV>, dim3(nwg), dim3(kWG), 0, s, g, c->d_tab, c->ord, c->lmax, n, idx, out); break;
    case STBEM_DK: hipLaunchKernelGGL(k_entries<OP_DK>, dim3(nwg), dim3(kWG), 0, s, g, c->d_tab, c->ord, c->lmax, n, idx, out); break;
    default: return fail(c, STBEM_EINVAL, "stbem_entries supports V, K, D, dV, dK");
    }
    HIPCHK(c, hipGetLastError());
    return STBEM_OK;
}

}  // extern "C"
