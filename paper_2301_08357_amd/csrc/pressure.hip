// Matrix-free P1 pressure operator and conjugate-gradient solver for
// AMD Instinct MI355X (gfx950).
//
// Operator (paper Sec. 3.4, weak problem of the projection stage, stiffness
// sign '+', consistent mass; Dirichlet pressure nodes of Sec. 3.6 eliminated
// symmetrically):  A_D = P_I (alpha M + beta K_c) P_I + P_B.
//
// Element formulas used by the kernels.  For a simplex with vertices X_0..X_d
// let e_k = X_k - X_0 and let n_k be row k of adj(J), J = [e_1 .. e_d]
// (3D: n_1 = e_2 x e_3, n_2 = e_3 x e_1, n_3 = e_1 x e_2; 2D: n_1 = (e2y, -e2x),
// n_2 = (-e1y, e1x)), det = e_1 . n_1 > 0 after orientation.  Then
// grad(phi_k) = n_k / det, |T| = det / d!, and for nodal values x_0..x_d
//     G   = sum_k n_k (x_k - x_0)                 (= det * grad x_h)
//     (K x)_k = c |T| grad(phi_k) . grad(x_h) = w n_k . G,  w = c / (d! det)
//     (K x)_0 = -sum_k (K x)_k
//     (M x)_a = |T| / ((d+1)(d+2)) * (x_a + sum_b x_b)
// (evaluated as fma(m, x_a, m * sum_b x_b) with m = |T| / ((d+1)(d+2))).
// The per-element factor beta * c_e / (d! det_e) is precomputed; the geometry
// is recomputed from the vertex coordinates on every apply.
//
// Determinism: every node sums its element contributions in ascending
// element order (both apply kernels use the same order and the same
// arithmetic, so they agree bit for bit), and every dot product is a fixed
// tree inside each block followed by a sum of the block partials in block
// order.  That last sum is done redundantly by every block of the kernel
// that consumes it, so the solver needs no atomics and no grid-wide fences;
// results are bitwise reproducible run to run.
//
// One CG iteration k is two kernels:
//   apply(k):  [prologue: rr_{k-1}, beta, convergence test]
//              p_k = r_{k-1} + beta p_{k-1} (formed while staging), q = A p_k,
//              block partials of p_k . q
//   update(k): [prologue: alpha = rr_{k-1} / p_k.q, breakdown test]
//              x += alpha p_k, r -= alpha q, block partials of r.r
// The partials of r.r alternate between two buffers by iteration parity, and
// p alternates between two buffers, so no kernel overwrites data that another
// block of the same kernel still reads.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "layout.hpp"
#include "pressure_cg.h"

namespace {

constexpr int BLK = 256;
constexpr int VGRID_MAX = 1024;      // blocks of the vector kernels
constexpr int AGRID_MAX = 2048;      // blocks of the tiled apply
constexpr uint32_t DIR_BIT = 0x80000000u;

struct CGState {
    double bnorm;    // ||rhs||
    double tol;      // rtol * ||rhs||
    double rr;       // r.r at the last completed iteration
    double tt;       // ||rhs - A x||^2 (true residual)
    int32_t iter;    // completed iterations
    int32_t max_iter;
    int32_t done;
    int32_t status;
    int32_t k_first; // launch index of this solve's first iteration (batched solves)
    int32_t pad;
};

// ------------------------------------------------------------------ reductions

// Lane moves for the wave sum, on the two 32-bit halves of a double.
// lanes_down32: lane l < 32 receives lane l + 32 (v_permlane32_swap);
// lanes_down16: lane l of rows 0 and 2 receives lane l + 16
// (v_permlane16_swap); row_down<N>: lane l receives lane l + N of its row
// of 16 (DPP row_shl, N < 16).  Other lanes receive values the sum does
// not use.
__device__ __forceinline__ double lanes_down32(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap(unsigned(b), unsigned(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(unsigned(b >> 32), unsigned(b >> 32), false, false);
    return __longlong_as_double((long long)((unsigned long long)hi[1] << 32 | lo[1]));
}

__device__ __forceinline__ double lanes_down16(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap(unsigned(b), unsigned(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(unsigned(b >> 32), unsigned(b >> 32), false, false);
    return __longlong_as_double((long long)((unsigned long long)hi[1] << 32 | lo[1]));
}

template <int N>
__device__ __forceinline__ double row_down(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), 0x100 + N, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), 0x100 + N, 0xf, 0xf, true);
    return __longlong_as_double((long long)((unsigned long long)unsigned(hi) << 32 | unsigned(lo)));
}

// Sum over the 64 lanes of a wave as a fixed tree: lane l adds lane l + 32,
// then l + 16, 8, 4, 2 and 1 (each step only needs the lanes below the
// stride).  The sum is in lane 0 only; the other lanes hold partial or
// meaningless values.  The lane moves are VALU operations, not LDS
// permutes, so the six steps cost a few dozen cycles.
__device__ inline double wave_sum(double v)
{
    v += lanes_down32(v);
    v += lanes_down16(v);
    v += row_down<8>(v);
    v += row_down<4>(v);
    v += row_down<2>(v);
    v += row_down<1>(v);
    return v;
}

// Lane 0's value of v in every lane (two scalar reads).
__device__ __forceinline__ double from_lane0(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane(unsigned(b), 0), hi = __builtin_amdgcn_readlane(unsigned(b >> 32), 0);
    return __longlong_as_double((long long)((unsigned long long)hi << 32 | lo));
}

// Block sum in a fixed order; the result is valid in every thread.  NTH is
// the block size; red holds NTH / 64 doubles.
template <int NTH = BLK>
__device__ inline double block_sum_all(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int k = 1; k < NTH / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// st->done as seen by thread 0, broadcast so the whole block takes the same branch.
__device__ inline bool block_done(const CGState *st)
{
    __shared__ int flag;
    if (threadIdx.x == 0) flag = st->done;
    __syncthreads();
    const bool d = flag != 0;
    __syncthreads();
    return d;
}

// Sum of n block partials, in the same fixed order in every block.  The
// first BLK threads do the summing whatever the block size NTH, so every
// kernel that sums the same partials gets the same bits (the lanes past BLK
// add exact zeros).
template <int NTH = BLK>
__device__ inline double sum_partials(const double *part, int n, double *red)
{
    double v = 0.0;
    if (threadIdx.x < BLK)
        for (int k = threadIdx.x; k < n; k += BLK) v += part[k];
    return block_sum_all<NTH>(v, red);
}

// ----------------------------------------------------------- element kernel

template <class R>
struct MeshT {
    int N, E;
    const int4 *conn;     // 4 vertex ids per element, bit 31 = Dirichlet vertex
    const R *X, *Y, *Z;
    const R *w;           // beta * c_e / (d! det_e), per element
    const uint8_t *dir;   // Dirichlet flag per node
    R mdiag, mfull;       // mass coefficients of x_a and of S = sum_b x_b, per unit det (elem_contrib)
    R per[3], iper[3];    // period and 1/period per axis; 0 = open axis
};
using Mesh = MeshT<double>;

// Edge vectors e[k-1] = x_k - x_0, k = 1..DIM, of one simplex.  With PER (a
// periodic mesh, whose matching boundary vertices are merged) each component
// takes its minimum image: the multiple of the period nearest to it is
// subtracted, which brings it into [-per/2, per/2].  Open axes carry
// per = iper = 0, for which the subtraction is an exact no-op; a wrapped
// component d, |d| in [per/2, 2 per], loses exactly one period.
template <int DIM, bool PER, class R>
__device__ __forceinline__ void elem_edges(const R *X, const R *Y, const R *Z, const MeshT<R> &g, R e[3][3])
{
#pragma unroll
    for (int k = 1; k <= DIM; ++k) {
        e[k - 1][0] = X[k] - X[0];
        e[k - 1][1] = Y[k] - Y[0];
        e[k - 1][2] = (DIM == 3) ? Z[k] - Z[0] : R(0);
        if (PER) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) e[k - 1][c] = fma(-g.per[c], rint(e[k - 1][c] * g.iper[c]), e[k - 1][c]);
        }
    }
}


// (alpha M_e + beta K_e) x_e for one simplex: out[a] for the local vertices.
// xv are the nodal values (zero for Dirichlet vertices), w the element factor.
// The mass part is det (mdiag x_a + mfull S), S = sum_b x_b: the consistent
// mass has mdiag = mfull = alpha / (d! (d+1) (d+2)) (|T| (1 + delta_ab) /
// ((d+1)(d+2))); the lumped mass (diagonal, |T| / (d+1) per vertex) has
// mdiag = alpha / (d! (d+1)) and mfull = 0.
template <int DIM, class R>
__device__ __forceinline__ void elem_contrib(const R e[3][3], const R *xv, R w, R mdiag, R mfull, R out[4])
{
    if (DIM == 2) {
        const R e1x = e[0][0], e1y = e[0][1];
        const R e2x = e[1][0], e2y = e[1][1];
        const R det = e1x * e2y - e1y * e2x;
        const R n1x = e2y, n1y = -e2x, n2x = -e1y, n2y = e1x;
        const R d1 = xv[1] - xv[0], d2 = xv[2] - xv[0];
        const R Gx = n1x * d1 + n2x * d2, Gy = n1y * d1 + n2y * d2;
        const R r1 = n1x * Gx + n1y * Gy;
        const R r2 = n2x * Gx + n2y * Gy;
        const R r0 = -(r1 + r2);
        const R S = xv[0] + xv[1] + xv[2];
        const R m = mdiag * det, mS = (mfull * det) * S;
        out[0] = fma(w, r0, fma(m, xv[0], mS));
        out[1] = fma(w, r1, fma(m, xv[1], mS));
        out[2] = fma(w, r2, fma(m, xv[2], mS));
        out[3] = R(0);
    } else {
        const R e1x = e[0][0], e1y = e[0][1], e1z = e[0][2];
        const R e2x = e[1][0], e2y = e[1][1], e2z = e[1][2];
        const R e3x = e[2][0], e3y = e[2][1], e3z = e[2][2];
        const R n1x = e2y * e3z - e2z * e3y, n1y = e2z * e3x - e2x * e3z, n1z = e2x * e3y - e2y * e3x;
        const R n2x = e3y * e1z - e3z * e1y, n2y = e3z * e1x - e3x * e1z, n2z = e3x * e1y - e3y * e1x;
        const R n3x = e1y * e2z - e1z * e2y, n3y = e1z * e2x - e1x * e2z, n3z = e1x * e2y - e1y * e2x;
        const R det = e1x * n1x + e1y * n1y + e1z * n1z;
        const R d1 = xv[1] - xv[0], d2 = xv[2] - xv[0], d3 = xv[3] - xv[0];
        const R Gx = n1x * d1 + n2x * d2 + n3x * d3;
        const R Gy = n1y * d1 + n2y * d2 + n3y * d3;
        const R Gz = n1z * d1 + n2z * d2 + n3z * d3;
        const R r1 = n1x * Gx + n1y * Gy + n1z * Gz;
        const R r2 = n2x * Gx + n2y * Gy + n2z * Gz;
        const R r3 = n3x * Gx + n3y * Gy + n3z * Gz;
        const R r0 = -(r1 + r2 + r3);
        const R S = xv[0] + xv[1] + xv[2] + xv[3];
        const R m = mdiag * det, mS = (mfull * det) * S;
        out[0] = fma(w, r0, fma(m, xv[0], mS));
        out[1] = fma(w, r1, fma(m, xv[1], mS));
        out[2] = fma(w, r2, fma(m, xv[2], mS));
        out[3] = fma(w, r3, fma(m, xv[3], mS));
    }
}

template <int DIM, class R>
__device__ __forceinline__ R elem_det(const R e[3][3])
{
    if (DIM == 2) {
        const R e1x = e[0][0], e1y = e[0][1];
        const R e2x = e[1][0], e2y = e[1][1];
        return e1x * e2y - e1y * e2x;
    }
    const R e1x = e[0][0], e1y = e[0][1], e1z = e[0][2];
    const R e2x = e[1][0], e2y = e[1][1], e2z = e[1][2];
    const R e3x = e[2][0], e3y = e[2][1], e3z = e[2][2];
    const R n1x = e2y * e3z - e2z * e3y, n1y = e2z * e3x - e2x * e3z, n1z = e2x * e3y - e2y * e3x;
    return e1x * n1x + e1y * n1y + e1z * n1z;
}


// w_e = beta * c_e / (d! det_e)
template <int DIM, class R, bool PER>
__global__ void __launch_bounds__(BLK) k_factors(MeshT<R> g, const double *__restrict__ coef, double beta,
                                                 R *__restrict__ w)
{
    const int e = blockIdx.x * BLK + threadIdx.x;
    if (e >= g.E) return;
    const int4 c = g.conn[e];
    const int v[4] = {c.x & 0x7fffffff, c.y & 0x7fffffff, c.z & 0x7fffffff, c.w & 0x7fffffff};
    R X[4], Y[4], Z[4];
    for (int a = 0; a <= DIM; ++a) {
        X[a] = g.X[v[a]];
        Y[a] = g.Y[v[a]];
        Z[a] = (DIM == 3) ? g.Z[v[a]] : R(0);
    }
    R ed[3][3];
    elem_edges<DIM, PER>(X, Y, Z, g, ed);
    const R fact = (DIM == 2) ? R(2) : R(6);
    w[e] = R(beta * coef[e]) / (fact * elem_det<DIM, R>(ed));
}

// per-instance copy of the element factor, for the tiled apply
template <class R>
__global__ void __launch_bounds__(BLK) k_inst_factors(int n, const int *__restrict__ inst_elem,
                                                      const R *__restrict__ w, R *__restrict__ iw)
{
    const int j = blockIdx.x * BLK + threadIdx.x;
    if (j < n) iw[j] = w[inst_elem[j]];
}

// ------------------------------------------------------------- CG plumbing

// Arguments of one CG iteration (k >= 1).  With first set, beta = 0.
template <class R>
struct IterT {
    int k;
    int first;
    const R *r;
    const R *p_old;        // p_{k-1}
    R *p_new;              // p_k
    R *q;                  // A p_k
    CGState *st;
    double *hist;
    double *part_pq;       // apply partials (n_apply_blocks)
    const double *rr_cur;  // partials of r_{k-1}.r_{k-1}
    const double *rr_prev; // partials of r_{k-2}.r_{k-2}
    int n_vblocks;
};
using Iter = IterT<double>;

// Prologue of apply(k): every block sums the partials of r_{k-1}.r_{k-1}
// (and of the previous one for beta) and takes the convergence decision;
// block 0 records it.  Returns false when the iteration must not run.
// iter_decide is the part after the test of st->done.
template <class R, int NTH = BLK>
__device__ inline bool iter_decide(const IterT<R> &it, double *red, double &beta, int vb)
{
    const double rr = sum_partials<NTH>(it.rr_cur, it.n_vblocks, red);
    beta = 0.0;
    if (!it.first) beta = rr / sum_partials<NTH>(it.rr_prev, it.n_vblocks, red);
    const double nr = sqrt(rr);
    const bool bad = !isfinite(rr);
    const bool stop = bad || !(nr > it.st->tol) || (it.k - 1) >= it.st->max_iter;
    if (vb == 0 && threadIdx.x == 0) {
        if (!(it.first && it.k > 1)) it.hist[it.k - 1] = nr / it.st->bnorm;
        it.st->iter = it.k - 1;
        it.st->rr = rr;
        if (bad) it.st->status = PM_EBREAKDOWN;
        if (stop) it.st->done = 1;
    }
    return !stop;
}

template <class R>
__device__ inline bool iter_prologue(const IterT<R> &it, double *red, double &beta, int vb)
{
    if (block_done(it.st)) return false;
    return iter_decide(it, red, beta, vb);
}

// Tile schedule: workgroups are dispatched round-robin over the 8 XCDs
// (block b runs on XCD b mod 8), and each XCD has its own L2.  Block b takes
// the tiles of XCD b mod 8's contiguous share of the Morton order, so blocks
// running side by side on one XCD work on neighbouring tiles and share their
// halo nodes in that L2.  tile_at(b, k) is the k-th tile of block b, or -1.
constexpr int N_XCD = 8;

__device__ __forceinline__ int tile_at(int b, int k, int n_blocks, int n_tiles)
{
    if (n_blocks < N_XCD || (n_blocks % N_XCD) != 0) {
        const int t = b + k * n_blocks;
        return t < n_tiles ? t : -1;
    }
    const int per_xcd_blocks = n_blocks / N_XCD;
    const int share = (n_tiles + N_XCD - 1) / N_XCD;
    const int x = b % N_XCD, j = b / N_XCD;
    const int t = x * share + j + k * per_xcd_blocks;
    const int end = min((x + 1) * share, n_tiles);
    return t < end ? t : -1;
}

// The block index a one-item-per-lane kernel works on, chosen so that XCD
// x = b mod 8 runs a contiguous chunk of the index range (blocks x, x + 8,
// ... take chunk x in order): items that share gathered data then share
// one L2.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b % N_XCD, j = b / N_XCD;
    const int q = nb / N_XCD, r = nb % N_XCD;
    return x * q + min(x, r) + j;
}

// ------------------------------------------------------------ apply kernels

// One lane per node: y_i = sum over the node's elements (ascending) of the
// element contribution to the node's local vertex; Dirichlet rows copy x.
// Reference kernel: each element is recomputed for each of its vertices.
// With CG set, x is p_k = r + beta p_{k-1}, formed on the fly.
// Nodes are visited in the tiled kernel's order (tile t by block t mod grid,
// node node_off[t] + j*BLK + lane), so the block partials of p.Ap, and hence
// whole solves, agree bit for bit between the two kernels.
template <int DIM, bool CG, bool PER>
__global__ void __launch_bounds__(BLK) k_apply_node(Mesh g, const int *__restrict__ off,
                                                    const int *__restrict__ ent, const int *__restrict__ node_off,
                                                    int n_tiles, const double *__restrict__ x,
                                                    double *__restrict__ y, Iter it)
{
    __shared__ double red[BLK / 64];
    double beta = 0.0;
    if (CG && !iter_prologue(it, red, beta, int(blockIdx.x))) return;
    auto val = [&](int v) -> double {
        if (!CG) return x[v];
        return it.first ? it.r[v] : it.r[v] + beta * it.p_old[v];
    };
    double part = 0.0;
    for (int kt = 0;; ++kt) {
    const int t = tile_at(blockIdx.x, kt, gridDim.x, n_tiles);
    if (t < 0) break;
    const int ts = node_off[t], te = node_off[t + 1];
    for (int jj = threadIdx.x; ts + jj < te; jj += BLK) {
        const int i = ts + jj;
        const double xi = val(i);
        double yi = 0.0;
        if (g.dir[i]) {
            yi = xi;
        } else {
            for (int k = off[i]; k < off[i + 1]; ++k) {
                const int en = ent[k];
                const int4 c = g.conn[en >> 2];
                const int cv[4] = {c.x, c.y, c.z, c.w};
                double X[4], Y[4], Z[4], xv[4], o[4];
                for (int a = 0; a <= DIM; ++a) {
                    const int v = cv[a] & 0x7fffffff;
                    X[a] = g.X[v];
                    Y[a] = g.Y[v];
                    Z[a] = (DIM == 3) ? g.Z[v] : 0.0;
                    xv[a] = (cv[a] < 0) ? 0.0 : val(v);
                }
                if (DIM == 2) xv[3] = 0.0;
                double ed[3][3];
                elem_edges<DIM, PER>(X, Y, Z, g, ed);
                elem_contrib<DIM, double>(ed, xv, g.w[en >> 2], g.mdiag, g.mfull, o);
                const int a = en & 3;
                yi += (a == 0) ? o[0] : (a == 1) ? o[1] : (a == 2) ? o[2] : o[3];
            }
        }
        y[i] = yi;
        if (CG) {
            it.p_new[i] = xi;
            part += xi * yi;
        }
    }
    }
    if (CG) {
        const double bs = block_sum_all(part, red);
        if (threadIdx.x == 0) it.part_pq[blockIdx.x] = bs;
    }
}

// Tile-local instance record: 4 x 16 bits, vertex a in bits 16a..16a+15 of
// the (x, y) pair; the low LVB bits are the vertex's local index (own node
// i -> i - first node of the tile, halo node -> T + rank in the tile's halo
// list), the high bits its row (rank of the element among the own node's
// elements, ascending element id).  Halo vertices carry the row max_deg,
// an extra row of the sums table that no node reads, so every vertex's
// contribution is written to row * RS + (local index mod T) without a test;
// the unused fourth vertex of a triangle is 0 and never processed.
template <int T>
struct TileGeom {
    static_assert(T == 128 || T == 256 || T == 512, "tile sizes are powers of two");
    static constexpr int LVB = (T <= 256) ? 10 : 11;       // bits of a local index
    static constexpr unsigned LV_MASK = (1u << LVB) - 1u;
    static constexpr int MAX_ROWS = 1 << (16 - LVB);       // rows a record can name (incl. the extra row)
    static constexpr int MAX_LOCAL = 1 << LVB;             // own + halo nodes a record can name
    static constexpr int RS = T + 1;                       // row stride of the sums table (padded)
};

// Size classes of the tiled kernel: (tile nodes, instances per lane,
// node-table entries, threads per block).  Setup picks the first class of
// the tile size that covers the largest tile's instance count and node
// table.  256-node tiles run 512 threads: two such blocks fill a CU's LDS
// with the same 16 waves as four 128-node blocks.
struct TileClass {
    int t, ipt, lm, nth;
};
constexpr TileClass TILE_CLASSES[] = {
    {128, 2, 256, 256},   {128, 4, 256, 256},   {128, 4, 384, 256},  {128, 6, 448, 256},  {128, 8, 512, 256},
    {128, 12, 768, 256},  {256, 3, 512, 512},   {256, 4, 768, 512},  {256, 6, 768, 512},  {256, 8, 1024, 512},
    {512, 16, 1024, 256}, {512, 20, 1536, 256}, {512, 24, 2048, 256}};
constexpr int N_TILE_CLASSES = sizeof(TILE_CLASSES) / sizeof(TILE_CLASSES[0]);

template <class R>
struct TileArgsT {
    int n_tiles;
    int max_deg;                  // rows of the LDS sums table
    const int *node_off;          // tile t owns nodes [node_off[t], node_off[t+1])
    const int *halo_off, *halo;   // halo node ids, Dirichlet flag in bit 31
    const int *inst_off;
    const uint2 *inst;            // packed instance records
    const R *inst_w;              // element factor per instance
    const uint8_t *nflag;         // per node: element count | Dirichlet << 7 (read for own nodes)
};

// LDS bytes of the tiled kernel: node table (DIM+1 fields of LM entries)
// and the sums table (max_deg rows of RS plus the row of halo writes).
template <class R, int T>
constexpr size_t tile_lds_bytes(int dim, int lm, int max_deg)
{
    return sizeof(R) * (size_t(dim + 1) * size_t(lm) + size_t(max_deg + 1) * TileGeom<T>::RS);
}

// Morton-tiled apply.  Each block walks its tiles (tile_at); for every tile
//  1. the coordinates and nodal values of the tile's own and halo nodes go
//     to the LDS node table (Dirichlet values as 0); under CG the value is
//     p_k = r + beta p_{k-1} and the block stores p_k for its own nodes;
//  2. each lane computes whole elements (its instances, held in registers)
//     from the node table and writes the contribution to each own vertex i
//     into S[row][i], row = rank of the element among node i's elements
//     (writes for halo vertices go to a sink);
//  3. each own node sums S[0..deg-1][i] in row order (ascending element id).
// Every element is computed once per tile that contains one of its vertices.
// The loads of tile k+1 are issued while tile k is processed: its offsets
// one tile earlier, its halo ids at tile k's staging, its node data as tile
// k's element phase starts and its instances slot by slot during it, so
// their latency overlaps tile k's work and that of the other blocks of the
// CU.  IPT instances per lane and LM node-table entries cover the largest
// tile (checked at setup).  Own node l of the tile is staged by lane
// l mod BLK in slot l / BLK, which is also the lane that sums its row, so the
// own values stay in registers between the phases.
// The body runs as virtual block vb of nvb (a real block of a single-mesh
// launch, or one (mesh, slot) pair of a batched launch).
template <int DIM, bool CG, class R, int T, int IPT, int LM, int NTH, bool PER>
__device__ __forceinline__ void apply_tiled_body(const MeshT<R> &g, const TileArgsT<R> &ta,
                                                 const R *__restrict__ x, R *__restrict__ y, const IterT<R> &it,
                                                 R *smem, double *red, int vb, int nvb)
{
    using G = TileGeom<T>;
    constexpr int NPT = (T + NTH - 1) / NTH, SPT = (LM + NTH - 1) / NTH, NF = DIM + 1, RS = G::RS;
    static_assert(LM >= T && LM <= G::MAX_LOCAL, "node table");
    if (CG && block_done(it.st)) return;
    R *const sN = smem;                      // NF x LM: X, Y, (Z,) value
    R *const sS = smem + NF * LM;            // (max_deg + 1) x RS sums

    // -- loads of one tile, into registers (under CG: r and p_{k-1}; p_k is
    // formed when staging, once beta is known)
    int gidx[SPT];
    uint2 ic[IPT];
    R iw[IPT];
    R vX[SPT], vY[SPT], vZ[SPT], vP[SPT], vQ[SPT];
    uint8_t vF[SPT];
    auto load_ids = [&](int s, int nt, int h0, int nh, int *gi) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int l = threadIdx.x + q * NTH;
            gi[q] = -1;
            if (l < nt) gi[q] = s + l;
            else if (l >= T && l < T + nh) gi[q] = ta.halo[h0 + l - T];
        }
    };
    // instance records and factors are read once per apply: non-temporal
    // loads keep them from evicting node data that neighbouring tiles
    // read again as halo
    auto load_inst = [&](int k, int i0, int ni) {
        const int j = threadIdx.x + k * NTH;
        if (j < ni) {
            const unsigned long long raw =
                __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(ta.inst) + (i0 + j));
            ic[k] = make_uint2(unsigned(raw), unsigned(raw >> 32));
            iw[k] = __builtin_nontemporal_load(ta.inst_w + (i0 + j));
        }
    };
    // own slots (l < T) take the node's flag byte; halo slots take the
    // Dirichlet flag from bit 31 of the halo id (one gather fewer per halo node)
    auto load_nodes = [&](const int *gi) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int raw = gi[q];
            const int v = raw & 0x7fffffff;
            if (raw != -1) {
                vX[q] = g.X[v];
                vY[q] = g.Y[v];
                if (DIM == 3) vZ[q] = g.Z[v];
                if (CG) {
                    vP[q] = it.r[v];
                    vQ[q] = it.first ? R(0) : it.p_old[v];
                } else {
                    vP[q] = x[v];
                }
                const int l = threadIdx.x + q * NTH;
                vF[q] = (l < T) ? ta.nflag[v] : ((raw < 0) ? uint8_t(0x80) : uint8_t(0));
            }
        }
    };

    double part = 0.0;
    // offsets of tile tt as vector loads (lanes 0-5 of each wave: halo,
    // instance and node ranges), read out with readlane when needed: unlike
    // scalar loads they do not hold up the waits on LDS operations
    const int lane = threadIdx.x & 63;
    auto load_offsets = [&](int tt) -> int {
        int v = 0;
        if (tt >= 0 && lane < 6)
            v = (lane < 2) ? ta.halo_off[tt + lane] : (lane < 4) ? ta.inst_off[tt + lane - 2] : ta.node_off[tt + lane - 4];
        return v;
    };
    int t = tile_at(vb, 0, nvb, ta.n_tiles);
    int ni = 0, cs = 0, cn = 0;   // instances, first node and node count of tile t
    if (t >= 0) {
        const int h0 = ta.halo_off[t], nh = ta.halo_off[t + 1] - h0;
        const int i0 = ta.inst_off[t];
        ni = ta.inst_off[t + 1] - i0;
        cs = ta.node_off[t];
        cn = ta.node_off[t + 1] - cs;
        load_ids(cs, cn, h0, nh, gidx);
#pragma unroll
        for (int k = 0; k < IPT; ++k) load_inst(k, i0, ni);
        load_nodes(gidx);
    }
    int tn = tile_at(vb, 1, nvb, ta.n_tiles);
    int vo = load_offsets(tn);
    // the sums of the prologue run while the first tile's loads are in flight
    double beta = 0.0;
    if (CG && !iter_decide<R, NTH>(it, red, beta, vb)) return;
    const R rbeta = R(beta);
    for (int kt = 0; t >= 0; ++kt) {
        const int s = cs, nt = cn;
        // 1. node table; own values kept for the row sums
        R ownP[NPT];
        uint8_t ownF[NPT];
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int l = threadIdx.x + q * NTH;
            if (CG && !it.first) vP[q] = vP[q] + rbeta * vQ[q];   // p_k = r + beta p_{k-1}
            if (gidx[q] != -1) {
                const bool d = (vF[q] & 0x80u) != 0;
                sN[l] = vX[q];
                sN[LM + l] = vY[q];
                if (DIM == 3) sN[2 * LM + l] = vZ[q];
                sN[(NF - 1) * LM + l] = d ? R(0) : vP[q];
                if (CG && l < nt) it.p_new[gidx[q]] = vP[q];
            }
            if (q < NPT) {
                ownP[q] = vP[q];
                ownF[q] = vF[q];
            }
        }
        // offsets and halo ids of the next tile
        const int h0n = __builtin_amdgcn_readlane(vo, 0), nhn = __builtin_amdgcn_readlane(vo, 1) - h0n;
        const int i0n = __builtin_amdgcn_readlane(vo, 2), nin = __builtin_amdgcn_readlane(vo, 3) - i0n;
        const int sn = __builtin_amdgcn_readlane(vo, 4), cnn = __builtin_amdgcn_readlane(vo, 5) - sn;
        int gidn[SPT];
        if (tn >= 0) load_ids(sn, cnn, h0n, nhn, gidn);
        __syncthreads();
        // 2. element contributions into the sums table.  The next tile's
        // loads go into the registers as this tile frees them: its node
        // data at once (the staging above freed those registers), its
        // instances slot by slot.  The waves run this phase at raised
        // priority, so that the issue slots of a SIMD go to the element
        // work of whichever block is in it, while the other phases mostly
        // wait on LDS and memory.
        if (tn >= 0) {
#pragma unroll
            for (int q = 0; q < SPT; ++q) gidx[q] = gidn[q];
            load_nodes(gidx);
        }
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const int j = threadIdx.x + k * NTH;
            if (j < ni) {
                const unsigned u[4] = {ic[k].x & 0xffffu, ic[k].x >> 16, ic[k].y & 0xffffu, ic[k].y >> 16};
                R X[4], Y[4], Z[4], xv[4], o[4];
#pragma unroll
                for (int a = 0; a <= DIM; ++a) {
                    const int lv = int(u[a] & G::LV_MASK);
                    X[a] = sN[lv];
                    Y[a] = sN[LM + lv];
                    Z[a] = (DIM == 3) ? sN[2 * LM + lv] : R(0);
                    xv[a] = sN[(NF - 1) * LM + lv];
                }
                if (DIM == 2) xv[3] = R(0);
                R ed[3][3];
                elem_edges<DIM, PER>(X, Y, Z, g, ed);
                elem_contrib<DIM, R>(ed, xv, iw[k], g.mdiag, g.mfull, o);
#pragma unroll
                for (int a = 0; a <= DIM; ++a)
                    sS[int(u[a] >> G::LVB) * RS + int(u[a] & unsigned(T - 1))] = o[a];
            }
            if (tn >= 0) load_inst(k, i0n, nin);
        }
        __builtin_amdgcn_s_setprio(0);
        const int tn2 = (tn >= 0) ? tile_at(vb, kt + 2, nvb, ta.n_tiles) : -1;
        vo = load_offsets(tn2);
        __syncthreads();
        // 3. row sums in ascending element order
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int l = threadIdx.x + j * NTH;
            if (l < nt) {
                const int d = ownF[j] & 0x7f;
                R yi = R(0);
                // rows in chunks of 8: the reads of a chunk are issued together
                for (int k0 = 0; k0 < d; k0 += 8) {
                    R v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < d) v[u] = sS[(k0 + u) * RS + l];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < d) yi += v[u];
                }
                // Dirichlet rows: y = x (p_k under CG)
                if (ownF[j] & 0x80u) yi = ownP[j];
                if (CG) part += double(ownP[j]) * double(yi);
                y[s + l] = yi;
            }
        }
        t = tn;
        ni = nin;
        cs = sn;
        cn = cnn;
        tn = tn2;
    }
    if (CG) {
        const double bs = block_sum_all<NTH>(part, red);
        if (threadIdx.x == 0) it.part_pq[vb] = bs;
    }
}

// Waves per SIMD the register budget is held to: four for the FP64 classes
// whose LDS tables admit four blocks per CU (128-node tiles, node table
// <= 448).  The FP32 kernels fit five waves without a bound (forcing six
// spills registers and was measured slower).
template <class R, int T, int LM>
constexpr int tile_waves()
{
    return (sizeof(R) == 8 && ((T == 128 && LM <= 448) || (T == 256 && LM <= 768))) ? 4 : 1;
}

template <int DIM, bool CG, class R, int T, int IPT, int LM, int NTH, bool PER>
__global__ void __launch_bounds__(NTH, (tile_waves<R, T, LM>())) k_apply_tiled(MeshT<R> g, TileArgsT<R> ta,
                                                                             const R *__restrict__ x,
                                                                             R *__restrict__ y, IterT<R> it)
{
    extern __shared__ double smem_d[];
    __shared__ double red[NTH / 64];
    apply_tiled_body<DIM, CG, R, T, IPT, LM, NTH, PER>(g, ta, x, y, it, reinterpret_cast<R *>(smem_d), red,
                                                       int(blockIdx.x), int(gridDim.x));
}

// ------------------------------------------------------------- CG vectors

// ------------------------------------------- one-launch solve of a small mesh

constexpr int SMALL_NTH = 1024;   // one workgroup
// elements per lane: E <= 4096 triangles or 3072 tetrahedra
constexpr int small_ept(int dim) { return dim == 2 ? 4 : 3; }
// With at most two triangles per lane (E <= 2048) the lanes also keep
// their elements' edge vectors in registers, so the element phase reads
// only the operand from LDS (tetrahedra would spill).
constexpr int SMALL_GEO_EPT = 2;
constexpr int SMALL_MPT = 4;      // nodes per lane of the update (N <= 4 * 256 * n_vblocks)

// Bytes of dynamic LDS the one-launch solve needs (see k_solve_small).
inline size_t small_lds_bytes(int dim, int64_t N, int64_t E, int n_ablocks, int n_tiles)
{
    const size_t dbl = size_t(dim + 4) * size_t(N) + size_t(dim + 1) * size_t(E) + 2 * size_t(n_ablocks) + 16;
    return 8 * dbl + 4 * (size_t(N) + 1 + size_t(n_tiles) + 1) + size_t(N);
}

// Sum over one wave as a 256-lane block_sum_all forms it when the other
// three waves hold zeros: this wave's sum, then three zero wave sums.  The
// result (formed in lane 0, where wave_sum is exact) goes to every lane.
__device__ __forceinline__ double wave_as_block(double v)
{
    double s = wave_sum(v);
    s += 0.0;
    s += 0.0;
    s += 0.0;
    return from_lane0(s);
}

// Arguments of the one-launch solve (vectors in internal node order).
struct SmallArgs {
    const int *n2e_off, *n2e_ent;   // node-to-element lists (entries 4e + a)
    const int *node_off;            // tile t owns nodes [node_off[t], node_off[t+1])
    const int *new2old;             // internal -> caller node order
    int n_tiles, n_ablocks, n_vblocks;
    double *x, *r, *b;
    CGState *st;
    double *hist;
    double *rr_parts;               // r.r partials of parity 0; parity 1 at + VGRID_MAX
    int k0;                         // first iteration of this launch
    const double *rhs, *x0;         // with rhs set (k0 = 1): form b, x, r and the state first
    double rtol;
    int max_iter;
    double *hist_host;              // pinned host memory or null: the history, also written here
    CGState *st_host;               // pinned host memory or null: the final state, copied here
};

// A CG solve of a small mesh in one launch of one 1024-lane workgroup.
// With a.rhs set it starts the solve (the gather of rhs and x0, ||rhs||
// and the state, r = b - A x0); then it runs iterations from a.k0 (a start
// or a restart: beta = 0) until the stop, and if the solve stopped
// without a failure it forms the true residual b - A x of the final
// iterate, its norm in st->tt and its partials for a restart.  The
// coordinates, the node values and the element contributions live in LDS;
// each lane keeps its elements (vertex ids, contribution slots, factor) and
// the residual at its vector nodes in registers for the whole solve.  An
// iteration is five phases between block barriers: the direction update,
// the element contributions, the node sums with the p.q partials, p.q and
// alpha in wave 0, and the vector update with the r.r partials.  With
// a.hist_host and a.st_host set the history and, at the end, the state are
// written to those host buffers as well.
// The arithmetic is that of the multi-launch solve (k_prepare, k_begin,
// the apply, k_start, the two-kernel iteration, k_true_residual and
// k_finish_tt), operation for operation and in the same order, reductions
// included, so x, r, b, the iteration count, the history and the state
// equal the multi-launch solve's bit for bit:
//  - a node sums its element contributions in ascending element order
//    (its slots in the contribution table are its node-to-element list);
//  - the p.q partial of apply block vb is formed as that block forms it,
//    one tile per block, own node l of the tile in lane l of a 256-lane
//    block (waves 2 and 3 of it hold zeros): here one wave sums each half
//    of a tile, and the halves and zeros are added in the block's order;
//  - the vector lane tid takes nodes tid + m * 256 * n_vblocks, as lane
//    tid mod 256 of vector block tid / 256 does, and the four wave sums
//    of a vector block are added in order;
//  - the sums of partials are those of sum_partials in a 256-lane block,
//    which every wave forms for itself (in its lane 0, then broadcast).
// Requires one tile per apply block (at most 256 tiles of at most 128
// nodes), at most 4 vector blocks, N <= SMALL_MPT * 256 * n_vblocks and
// E <= EPT * 1024; the host checks all of it.  GEO: the edge vectors of
// the lane's elements stay in registers (the same values elem_edges forms
// from the node table in every apply otherwise).
template <int DIM, bool PER, int EPT, bool GEO>
__global__ void __launch_bounds__(SMALL_NTH) k_solve_small(Mesh g, SmallArgs a)
{
    extern __shared__ double sm[];
    const int N = g.N, E = g.E, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n_tiles = a.n_tiles, n_ablocks = a.n_ablocks, n_vblocks = a.n_vblocks;
    const bool start = a.rhs != nullptr;
    constexpr int NV = DIM + 1;
    // node table: per node X, Y, (Z,) and the operand with Dirichlet
    // entries 0, so one address per vertex reaches all of them
    double *const sN = sm;
    double *const sp = sN + size_t(NV) * N, *const sq = sp + N, *const sx = sq + N;
    double *const sC = sx + N;                                        // NV * E contributions, by slot
    double *const sph = sC + size_t(NV) * E, *const sred = sph + 2 * n_ablocks;   // half-tile sums
    int *const sOff = reinterpret_cast<int *>(sred + 16);            // N + 1 slot offsets
    int *const sTo = sOff + N + 1;                                    // n_tiles + 1 tile offsets
    uint8_t *const sDir = reinterpret_cast<uint8_t *>(sTo + n_tiles + 1);
    int *const sInv = reinterpret_cast<int *>(sC);                    // setup only: slot of 4e + a

    __shared__ int done0;
    if (tid == 0) done0 = start ? 0 : a.st->done;
    for (int i = tid; i < N; i += SMALL_NTH) {
        sN[NV * i] = g.X[i];
        sN[NV * i + 1] = g.Y[i];
        if (DIM == 3) sN[NV * i + 2] = g.Z[i];
        sDir[i] = g.dir[i];
        const int j0 = a.n2e_off[i], j1 = a.n2e_off[i + 1];
        sOff[i] = j0;
        for (int j = j0; j < j1; ++j) sInv[a.n2e_ent[j]] = j;
    }
    if (tid == 0) sOff[N] = a.n2e_off[N];
    for (int t = tid; t <= n_tiles; t += SMALL_NTH) sTo[t] = a.node_off[t];
    // the vector nodes of this lane
    const int ustride = n_vblocks * BLK;
    auto unode = [&](int m) { return tid + m * ustride; };
    auto uvalid = [&](int m) { return tid < ustride && unode(m) < N; };
    double ur[SMALL_MPT];
    unsigned udir = 0;
    double v = 0.0;   // start: partial of rhs.rhs
#pragma unroll
    for (int m = 0; m < SMALL_MPT; ++m) {
        const int i = unode(m);
        ur[m] = 0.0;
        if (uvalid(m)) {
            if (g.dir[i]) udir |= 1u << m;
            if (start) {
                // k_prepare: gather rhs and x0; Dirichlet entries of x0 take rhs
                const int o = a.new2old[i];
                const double bi = a.rhs[o];
                double xi = a.x0 ? a.x0[o] : 0.0;
                if ((udir >> m) & 1u) xi = bi;
                a.b[i] = bi;
                sp[i] = bi;   // b until the first direction
                sx[i] = xi;
                v += bi * bi;
            } else {
                sx[i] = a.x[i];
                ur[m] = a.r[i];
            }
        }
    }
    if (start) {
        v = wave_sum(v);
        if (lane == 0) sred[wv] = v;
    }
    __syncthreads();
    // this lane's elements: vertex id (low 16 bits) and contribution slot
    // (high 16 bits) per vertex, and the element factor
    unsigned ev[EPT][NV];
    double ew[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * SMALL_NTH;
        ew[k] = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) ev[k][c] = 0;
        if (e < E) {
            const int4 c4 = g.conn[e];
            const int cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int c = 0; c < NV; ++c) ev[k][c] = unsigned(cv[c] & 0x7fffffff) | (unsigned(sInv[4 * e + c]) << 16);
            ew[k] = g.w[e];
        }
    }
    // sum_partials of the 256-lane blocks' sums of sred (n_vblocks blocks of 4 waves), in every lane
    auto vector_sum = [&]() {
        double u = 0.0;
        if (lane < n_vblocks) {
            double b4 = sred[4 * lane];
            b4 += sred[4 * lane + 1];
            b4 += sred[4 * lane + 2];
            b4 += sred[4 * lane + 3];
            u += b4;
        }
        return wave_as_block(u);
    };
    double tol, bnorm;
    int max_iter, status = 0;
    if (start) {
        // k_begin
        const double bb = vector_sum();
        bnorm = sqrt(bb);
        tol = a.rtol * bnorm;
        max_iter = a.max_iter;
        const bool ok = isfinite(bnorm), stop0 = !ok || !(bnorm > 0.0);
        status = ok ? 0 : PM_EINVAL;
        if (tid == 0) {
            CGState *st = a.st;
            st->bnorm = bnorm;
            st->tol = tol;
            st->rr = 0.0;
            st->tt = 0.0;
            st->iter = 0;
            st->max_iter = max_iter;
            st->status = ok ? 0 : PM_EINVAL;
            st->done = stop0 ? 1 : 0;
            st->k_first = 1;
            if (!(bnorm > 0.0)) {
                a.hist[0] = 0.0;
                if (a.hist_host) a.hist_host[0] = 0.0;
            }
            done0 = stop0 ? 1 : 0;
        }
    } else {
        tol = a.st->tol;
        bnorm = a.st->bnorm;
        max_iter = a.st->max_iter;
    }
    __syncthreads();   // sInv is read; sC takes contributions from here on
    double ged[GEO ? EPT : 1][3][3];
    if constexpr (GEO) {
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk) {
            double X[4] = {0.0, 0.0, 0.0, 0.0}, Y[4] = {0.0, 0.0, 0.0, 0.0}, Z[4] = {0.0, 0.0, 0.0, 0.0};
            if (tid + kk * SMALL_NTH < E) {
#pragma unroll
                for (int c = 0; c < NV; ++c) {
                    const double *nv = sN + NV * int(ev[kk][c] & 0xffffu);
                    X[c] = nv[0];
                    Y[c] = nv[1];
                    Z[c] = (DIM == 3) ? nv[2] : 0.0;
                }
            }
            elem_edges<DIM, PER>(X, Y, Z, g, ged[kk]);
        }
    }

    // The operator apply y = A v of the staged node values (Dirichlet
    // entries 0 in the node table, Dirichlet rows y = v): the element
    // contributions, then the node sums into sq.  With PART each half tile
    // stores the wave sum of its v.y terms in sph.
    auto apply = [&](const double *__restrict__ sv, bool part_on) {
        // The element records pass through an empty asm statement, so the
        // compiler forms their LDS addresses here instead of keeping one
        // register per address for the whole solve.
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk)
#pragma unroll
            for (int c = 0; c < NV; ++c) asm volatile("" : "+v"(ev[kk][c]));
#pragma unroll
        for (int kk = 0; kk < EPT; ++kk) {
            if (tid + kk * SMALL_NTH < E) {
                double xv[4], o[4];
                if constexpr (GEO) {
#pragma unroll
                    for (int c = 0; c < NV; ++c) xv[c] = sN[NV * int(ev[kk][c] & 0xffffu) + DIM];
                    if (DIM == 2) xv[3] = 0.0;
                    elem_contrib<DIM, double>(ged[kk], xv, ew[kk], g.mdiag, g.mfull, o);
                } else {
                    double X[4], Y[4], Z[4];
#pragma unroll
                    for (int c = 0; c < NV; ++c) {
                        const double *nv = sN + NV * int(ev[kk][c] & 0xffffu);
                        X[c] = nv[0];
                        Y[c] = nv[1];
                        Z[c] = (DIM == 3) ? nv[2] : 0.0;
                        xv[c] = nv[DIM];
                    }
                    if (DIM == 2) xv[3] = 0.0;
                    double ed[3][3];
                    elem_edges<DIM, PER>(X, Y, Z, g, ed);
                    elem_contrib<DIM, double>(ed, xv, ew[kk], g.mdiag, g.mfull, o);
                }
#pragma unroll
                for (int c = 0; c < NV; ++c) sC[ev[kk][c] >> 16] = o[c];
            }
        }
        __syncthreads();
        // A wave takes one half (64 nodes) of a tile; a half with no nodes
        // sums to +0, as the wave sum of zeros does.
        for (int hv = wv; hv < 2 * n_ablocks; hv += SMALL_NTH / 64) {
            const int t = tile_at(hv >> 1, 0, n_ablocks, n_tiles);
            const int s0 = (t >= 0) ? sTo[t] : 0, nt = (t >= 0) ? sTo[t + 1] - s0 : 0;
            const int l = lane + 64 * (hv & 1);
            double part = 0.0;
            if (l < nt) {
                const int i = s0 + l;
                const double vi = sv[i];
                double yi = 0.0;
                if (sDir[i]) {
                    yi = vi;
                } else {
                    // slots in chunks of 8: the reads of a chunk are issued together
                    const int j0 = sOff[i], d = sOff[i + 1] - j0;
                    for (int c = 0; c < d; c += 8) {
                        double cv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (c + u < d) cv[u] = sC[j0 + c + u];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (c + u < d) yi += cv[u];
                    }
                }
                sq[i] = yi;
                part += vi * yi;
            }
            if (part_on) {
                const double ws = wave_sum(part);
                if (lane == 0) sph[hv] = ws;
            }
        }
        __syncthreads();
    };
    // the node table's operand entries from x
    auto stage_x = [&]() {
        double xv[SMALL_MPT];
#pragma unroll
        for (int m = 0; m < SMALL_MPT; ++m) xv[m] = uvalid(m) ? sx[unode(m)] : 0.0;
#pragma unroll
        for (int m = 0; m < SMALL_MPT; ++m)
            if (uvalid(m)) sN[NV * unode(m) + DIM] = (udir >> m) & 1u ? 0.0 : xv[m];
        __syncthreads();
    };

    double rr = 0.0, rr_prev = 0.0;
    if (start) {
        // q = A x0; k_start: r = b - q (||rhs|| = 0 or not finite: x = 0,
        // r = 0), partials of r.r
        stage_x();
        apply(sx, false);
        const bool zero = !(bnorm > 0.0);
        double u = 0.0;
#pragma unroll
        for (int m = 0; m < SMALL_MPT; ++m)
            if (uvalid(m)) {
                const int i = unode(m);
                double ri = sp[i] - sq[i];
                if (zero) {
                    sx[i] = 0.0;
                    ri = 0.0;
                }
                ur[m] = ri;
                u += ri * ri;
            }
        u = wave_sum(u);
        if (lane == 0) sred[wv] = u;
        __syncthreads();
        rr = vector_sum();
    } else {
        double u = 0.0;
        if (lane < n_vblocks) u += a.rr_parts[((a.k0 - 1) & 1) * VGRID_MAX + lane];
        rr = wave_as_block(u);
    }
    int k = a.k0;
    bool first = true;
    // Every VALU instruction of a wave costs its SIMD four cycles, and one
    // workgroup is all the work there is, so work is kept off the waves
    // that do not need it: p.q and alpha are formed in wave 0 alone, whose
    // lane 0 passes them on through LDS, and the waves past the vector
    // blocks skip the vector phases.  The stopping decision and beta, from
    // rr, cost less in every wave than a barrier would.
    __shared__ double s_alpha;
    __shared__ int s_flag;   // set to 2 on a p.q breakdown
    if (tid == 0) s_flag = 0;
    __syncthreads();
    if (!done0) {
        for (;; ++k) {
            // the decision of the apply of iteration k (iter_decide), in every wave
            const double nr = sqrt(rr);
            const bool bad = !isfinite(rr);
            const bool stop = bad || !(nr > tol) || (k - 1) >= max_iter;
            if (tid == 0) {
                if (!(first && k > 1)) {
                    a.hist[k - 1] = nr / bnorm;
                    if (a.hist_host) a.hist_host[k - 1] = nr / bnorm;
                }
                a.st->iter = k - 1;
                a.st->rr = rr;
                if (bad) a.st->status = PM_EBREAKDOWN;
                if (stop) a.st->done = 1;
            }
            if (stop) {
                if (bad) status = PM_EBREAKDOWN;
                break;
            }
            const double beta = first ? 0.0 : rr / rr_prev;
            // 1. p_k = r + beta p_{k-1}.  Each phase reads all it needs
            // before it writes, so the reads of its items are issued
            // together (the LDS arrays share one base, and the compiler
            // would otherwise order each read after the previous item's
            // writes).
            if (tid < ustride) {   // whole waves
                double pv[SMALL_MPT];
#pragma unroll
                for (int m = 0; m < SMALL_MPT; ++m) pv[m] = (!first && uvalid(m)) ? sp[unode(m)] : 0.0;
#pragma unroll
                for (int m = 0; m < SMALL_MPT; ++m)
                    if (uvalid(m)) {
                        const int i = unode(m);
                        double pk = ur[m];
                        if (!first) pk = pk + beta * pv[m];
                        sp[i] = pk;
                        sN[NV * i + DIM] = (udir >> m) & 1u ? 0.0 : pk;
                    }
            }
            __syncthreads();
            // 2, 3. q = A p and the p.q partials of the apply blocks
            apply(sp, true);
            // 4. the update: alpha = rr / p.q, x += alpha p, r -= alpha q
            if (wv == 0) {
                double w4[4] = {0.0, 0.0, 0.0, 0.0};   // waves past the partials sum zeros
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u * 64 >= n_ablocks) break;
                    double pv = 0.0;
                    const int vb = u * 64 + lane;
                    if (vb < n_ablocks) {
                        // the partial of apply block vb: its two halves, then two zero waves
                        double bs = sph[2 * vb];
                        bs += sph[2 * vb + 1];
                        bs += 0.0;
                        bs += 0.0;
                        pv += bs;
                    }
                    w4[u] = wave_sum(pv);
                }
                if (lane == 0) {
                    double pq = w4[0];
                    pq += w4[1];
                    pq += w4[2];
                    pq += w4[3];
                    if (!(pq > 0.0) || !isfinite(pq)) {
                        a.st->status = PM_EBREAKDOWN;
                        a.st->done = 1;
                        s_flag = 2;
                    } else {
                        s_alpha = rr / pq;
                    }
                }
            }
            __syncthreads();
            if (s_flag) {
                status = PM_EBREAKDOWN;
                break;
            }
            const double alpha = s_alpha;
            double u = 0.0;
            if (tid < ustride) {   // whole waves
                double xv[SMALL_MPT], pv[SMALL_MPT], qv[SMALL_MPT];
#pragma unroll
                for (int m = 0; m < SMALL_MPT; ++m) {
                    xv[m] = pv[m] = qv[m] = 0.0;
                    if (uvalid(m)) {
                        const int i = unode(m);
                        xv[m] = sx[i];
                        pv[m] = sp[i];
                        qv[m] = sq[i];
                    }
                }
#pragma unroll
                for (int m = 0; m < SMALL_MPT; ++m)
                    if (uvalid(m)) {
                        sx[unode(m)] = xv[m] + alpha * pv[m];
                        const double ri = ur[m] - alpha * qv[m];
                        ur[m] = ri;
                        u += ri * ri;
                    }
            }
            if (tid < ustride) {
                u = wave_sum(u);
                if (lane == 0) sred[wv] = u;
            }
            __syncthreads();
            rr_prev = rr;
            rr = vector_sum();
            first = false;
        }
    }
    if (status == 0 && bnorm > 0.0) {
        // the true residual of the final iterate (launch_apply of x,
        // k_true_residual into the r.r partials of the final iteration's
        // parity, k_finish_tt)
        const int kdone = done0 ? a.st->iter : k - 1;
        stage_x();
        apply(sx, false);
        double u = 0.0;
#pragma unroll
        for (int m = 0; m < SMALL_MPT; ++m)
            if (uvalid(m)) {
                const int i = unode(m);
                const double ri = a.b[i] - sq[i];
                ur[m] = ri;
                u += ri * ri;
            }
        u = wave_sum(u);
        if (lane == 0) sred[wv] = u;
        __syncthreads();
        if (wv < n_vblocks && lane == 0) {
            double b4 = sred[4 * wv];
            b4 += sred[4 * wv + 1];
            b4 += sred[4 * wv + 2];
            b4 += sred[4 * wv + 3];
            a.rr_parts[(kdone & 1) * VGRID_MAX + wv] = b4;
        }
        if (wv == 0) {
            const double tt = vector_sum();
            if (tid == 0) a.st->tt = tt;
        }
    }
#pragma unroll
    for (int m = 0; m < SMALL_MPT; ++m)
        if (uvalid(m)) {
            a.x[unode(m)] = sx[unode(m)];
            a.r[unode(m)] = ur[m];
        }
    // every write to the state came from this lane, which reads them back
    if (tid == 0 && a.st_host) *a.st_host = *a.st;
}


// update(k): alpha = rr_{k-1} / p_k.q; x += alpha p_k; r -= alpha q;
// partials of r_k.r_k.  Runs as virtual block vb of nvb.
template <class R>
__device__ __forceinline__ void update_body(int N, R *__restrict__ x, R *__restrict__ r, const R *__restrict__ p,
                                            const R *__restrict__ q, CGState *st, const double *part_pq,
                                            int n_ablocks, const double *rr_cur, double *rr_out, double *red,
                                            int vb, int nvb)
{
    if (block_done(st)) return;
    // the lane's first PF nodes are loaded while the partials are summed
    constexpr int PF = 4;
    const int i0 = vb * BLK + threadIdx.x, stride = nvb * BLK;
    R vx[PF], vp[PF], vr[PF], vq[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = i0 + u * stride;
        if (i < N) {
            vx[u] = x[i];
            vp[u] = p[i];
            vr[u] = r[i];
            vq[u] = q[i];
        }
    }
    const double pq = sum_partials(part_pq, n_ablocks, red);
    const double rr = sum_partials(rr_cur, nvb, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (vb == 0 && threadIdx.x == 0) {
            st->status = PM_EBREAKDOWN;
            st->done = 1;
        }
        return;
    }
    const R a = R(rr / pq);
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = i0 + u * stride;
        if (i < N) {
            x[i] = vx[u] + a * vp[u];
            const R ri = vr[u] - a * vq[u];
            r[i] = ri;
            v += double(ri) * double(ri);
        }
    }
    for (int i = i0 + PF * stride; i < N; i += stride) {
        x[i] += a * p[i];
        const R ri = r[i] - a * q[i];
        r[i] = ri;
        v += double(ri) * double(ri);
    }
    const double bs = block_sum_all(v, red);
    if (threadIdx.x == 0) rr_out[vb] = bs;
}

template <class R>
__global__ void __launch_bounds__(BLK) k_update(int N, R *__restrict__ x, R *__restrict__ r,
                                                const R *__restrict__ p, const R *__restrict__ q,
                                                CGState *st, const double *part_pq, int n_ablocks,
                                                const double *rr_cur, int n_vblocks, double *rr_out)
{
    __shared__ double red[BLK / 64];
    (void)n_vblocks;
    update_body<R>(N, x, r, p, q, st, part_pq, n_ablocks, rr_cur, rr_out, red, int(blockIdx.x), int(gridDim.x));
}

// Gather the caller's rhs and initial guess into internal order; Dirichlet
// entries of the guess take the rhs value.  Partials of rhs.rhs.
__global__ void __launch_bounds__(BLK) k_prepare(int N, const int *__restrict__ new2old,
                                                 const uint8_t *__restrict__ dir,
                                                 const double *__restrict__ rhs,
                                                 const double *__restrict__ x0, double *__restrict__ b,
                                                 double *__restrict__ x, double *part)
{
    __shared__ double red[BLK / 64];
    double v = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) {
        const int o = new2old[i];
        const double bi = rhs[o];
        double xi = x0 ? x0[o] : 0.0;
        if (dir[i]) xi = bi;
        b[i] = bi;
        x[i] = xi;
        v += bi * bi;
    }
    const double bs = block_sum_all(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// One block: ||rhs|| and the solver state.
__global__ void __launch_bounds__(BLK) k_begin(CGState *st, const double *part, int n, double rtol,
                                               int max_iter, double *hist, int k_first)
{
    __shared__ double red[BLK / 64];
    const double bb = sum_partials(part, n, red);
    if (threadIdx.x == 0) {
        const double bn = sqrt(bb);
        st->bnorm = bn;
        st->tol = rtol * bn;
        st->rr = 0.0;
        st->tt = 0.0;
        st->iter = 0;
        st->max_iter = max_iter;
        st->status = isfinite(bn) ? 0 : PM_EINVAL;
        st->done = (!isfinite(bn) || !(bn > 0.0)) ? 1 : 0;
        st->k_first = k_first;
        if (!(bn > 0.0)) hist[0] = 0.0;
    }
}

// r = b - q (q = A x) and partials of r.r; rhs = 0 gives x = 0.
__global__ void __launch_bounds__(BLK) k_start(int N, const double *__restrict__ b,
                                               const double *__restrict__ q, double *__restrict__ x,
                                               double *__restrict__ r, const CGState *st, double *part)
{
    __shared__ double red[BLK / 64];
    const bool zero = !(st->bnorm > 0.0);
    double v = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) {
        double ri = b[i] - q[i];
        if (zero) {
            x[i] = 0.0;
            ri = 0.0;
        }
        r[i] = ri;
        v += ri * ri;
    }
    const double bs = block_sum_all(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// r = b - q (the true residual of x); partials of r.r.
__global__ void __launch_bounds__(BLK) k_true_residual(int N, const double *__restrict__ b,
                                                       const double *__restrict__ q,
                                                       double *__restrict__ r, double *part)
{
    __shared__ double red[BLK / 64];
    double v = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) {
        const double ri = b[i] - q[i];
        r[i] = ri;
        v += ri * ri;
    }
    const double bs = block_sum_all(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// One block: tt = sum of the partials; optionally reopen the solve.
__global__ void __launch_bounds__(BLK) k_finish_tt(CGState *st, const double *part, int n)
{
    __shared__ double red[BLK / 64];
    const double tt = sum_partials(part, n, red);
    if (threadIdx.x == 0) st->tt = tt;
}

__global__ void k_reopen(CGState *st)
{
    if (threadIdx.x == 0) st->done = 0;
}

// ------------------------------------------------- the space V_0 (Sec. 3.4)
// With no Dirichlet node and alpha = 0 the operator beta K_c is singular
// (its kernel is the constants) and the weak problem is posed in
// V_0 = {z : int z = 0}.  Testing with z in V_0 gives K p = b - (sum_i b_i /
// |Omega|) m, with m_i = int phi_i (the lumped mass weights, |Omega| =
// sum_i m_i), and the solution is the one with sum_i m_i p_i = 0.

// m_i = sum over node i's elements (ascending) of |T_e| / (d+1)
template <int DIM, bool PER>
__global__ void __launch_bounds__(BLK) k_lumped_mass(Mesh g, const int *__restrict__ off,
                                                     const int *__restrict__ ent, double *__restrict__ mw)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i >= g.N) return;
    constexpr double fact = (DIM == 2) ? 2.0 * 3.0 : 6.0 * 4.0;   // d! (d+1)
    double sum = 0.0;
    for (int k = off[i]; k < off[i + 1]; ++k) {
        const int4 c = g.conn[ent[k] >> 2];
        const int v[4] = {c.x & 0x7fffffff, c.y & 0x7fffffff, c.z & 0x7fffffff, c.w & 0x7fffffff};
        double X[4], Y[4], Z[4];
        for (int a = 0; a <= DIM; ++a) {
            X[a] = g.X[v[a]];
            Y[a] = g.Y[v[a]];
            Z[a] = (DIM == 3) ? g.Z[v[a]] : 0.0;
        }
        double ed[3][3];
        elem_edges<DIM, PER>(X, Y, Z, g, ed);
        sum += elem_det<DIM, double>(ed) / fact;
    }
    mw[i] = sum;
}

// block partials of sum_i w_i v_i (w = null: sum_i v_i)
__global__ void __launch_bounds__(BLK) k_wsum(int N, const double *__restrict__ w, const double *__restrict__ v,
                                              double *part)
{
    __shared__ double red[BLK / 64];
    double acc = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) acc += w ? w[i] * v[i] : v[i];
    const double bs = block_sum_all(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// v -= (sum of the n partials / denom) * (w ? w_i : 1); partials of v.v
// into bb (may be null)
__global__ void __launch_bounds__(BLK) k_sub_mean(int N, double *__restrict__ v, const double *__restrict__ w,
                                                  const double *part, int n, double denom, double *bb)
{
    __shared__ double red[BLK / 64];
    const double c = sum_partials(part, n, red) / denom;
    double acc = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) {
        const double vi = v[i] - c * (w ? w[i] : 1.0);
        v[i] = vi;
        acc += vi * vi;
    }
    if (bb) {
        const double bs = block_sum_all(acc, red);
        if (threadIdx.x == 0) bb[blockIdx.x] = bs;
    }
}

// -------------------------------------------------------- projection stage
// Sec. 3.3 - 3.5 around the solve.  Element data are in internal element
// order, dual-cell (face) data in the caller's face numbering.

struct ProjArgs {
    const int *efc;       // 4 per element: face opposite internal-local vertex a
    const int2 *fel;      // per face: internal elements (y = -1 on the boundary)
    const uint8_t *ebnd;  // per element: bit a set when the face opposite a is a boundary face
    const double *rho_f, *we_f, *wu_f, *bflux;
    double *erho, *ewe, *ewu, *erk, *evol, *egrad;   // per element (ewu, egrad: 3 each)
    double g1;            // gamma / (gamma - 1)
    double dt;
    double *w;            // element factors beta c_k / (d! det), written with c_k = H_k
};

// Corner ids and (minimum-image) edge vectors of element k.
template <int DIM, bool PER>
__device__ __forceinline__ void elem_corners(const Mesh &g, int k, int v[4], double ed[3][3])
{
    const int4 c = g.conn[k];
    v[0] = c.x & 0x7fffffff;
    v[1] = c.y & 0x7fffffff;
    v[2] = c.z & 0x7fffffff;
    v[3] = c.w & 0x7fffffff;
    double X[4], Y[4], Z[4];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        X[a] = g.X[v[a]];
        Y[a] = g.Y[v[a]];
        Z[a] = (DIM == 3) ? g.Z[v[a]] : 0.0;
    }
    elem_edges<DIM, PER>(X, Y, Z, g, ed);
}

// The same for vertex ids that are already known.
template <int DIM, bool PER>
__device__ __forceinline__ void elem_corners_of(const Mesh &g, const int v[4], double ed[3][3])
{
    double X[4], Y[4], Z[4];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        X[a] = g.X[v[a]];
        Y[a] = g.Y[v[a]];
        Z[a] = (DIM == 3) ? g.Z[v[a]] : 0.0;
    }
    elem_edges<DIM, PER>(X, Y, Z, g, ed);
}

// Adjugate normals n_a (grad phi_a = n_a / det; |n_a| = (d-1)! |face a|) and det.
template <int DIM>
__device__ __forceinline__ double elem_normals(const double ed[3][3], double n[4][3])
{
    if (DIM == 2) {
        n[1][0] = ed[1][1];
        n[1][1] = -ed[1][0];
        n[2][0] = -ed[0][1];
        n[2][1] = ed[0][0];
        n[1][2] = n[2][2] = 0.0;
    } else {
        const double(*e)[3] = ed;
        n[1][0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
        n[1][1] = e[1][2] * e[2][0] - e[1][0] * e[2][2];
        n[1][2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
        n[2][0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
        n[2][1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
        n[2][2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
        n[3][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
        n[3][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
        n[3][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double t = 0.0;
#pragma unroll
        for (int a = 1; a <= DIM; ++a) t += n[a][c];
        n[0][c] = -t;
    }
    return ed[0][0] * n[1][0] + ed[0][1] * n[1][1] + ed[0][2] * n[1][2];
}

// H_k = mean over the faces f of T_k of g1 P_f / rho_f, with P_f the mean of
// the face's vertex pressures pv (the face opposite vertex a has the others).
template <int DIM>
__device__ __forceinline__ double elem_enthalpy(const ProjArgs &pa, int k, const double pv[4])
{
    double h = 0.0;
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        double pf = 0.0;
#pragma unroll
        for (int b = 0; b <= DIM; ++b)
            if (b != a) pf += pv[b];
        pf /= double(DIM);
        h += pa.g1 * pf / pa.rho_f[pa.efc[4 * k + a]];
    }
    return h / double(DIM + 1);
}

// Right-hand side of the weak problem for one Picard iteration, the element
// part: contrib[4k + a] = the contribution of element k to its vertex a,
//   (W_E,k - (rho K)_k) |T_k|/(d+1) + dt H_k W_u,k . n_a / d!
//   - alpha (M_e P^n)_a - (A_e g)_a over the Dirichlet vertices
//   - dt bflux_f |f| / d for each boundary face f of T_k that holds vertex a.
// The node pass (k_proj_rhs_node) sums the contributions of each vertex.  It
// runs inside the kernel that has just formed H_k, w_k and (rho K)_k, so
// that the element's geometry and fields are read once.
template <int DIM>
__device__ __forceinline__ void rhs_elem_write(const Mesh &g, const ProjArgs &pa, int k, const int v[4],
                                               const double ed[3][3], const double n[4][3], double det,
                                               double wek, double rkk, const double u[3], double hk, double wk,
                                               const double pv[4], const double *__restrict__ gd,
                                               double *__restrict__ contrib)
{
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    const double vol = det / dfact;
    const double src = (wek - rkk) * (vol / double(DIM + 1));
    const double hdt = pa.dt * hk / dfact;
    const int4 c4 = g.conn[k];
    const int cv[4] = {c4.x, c4.y, c4.z, c4.w};
    double gv[4], o[4], t[4];
    double sp = 0.0;
    bool lift = false;
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        sp += pv[a];
        gv[a] = (cv[a] < 0) ? gd[v[a]] : 0.0;
        lift = lift || (cv[a] < 0);
    }
    if (DIM == 2) gv[3] = 0.0;
    if (lift) elem_contrib<DIM, double>(ed, gv, wk, g.mdiag, g.mfull, o);
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        double un = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) un += u[c] * n[a][c];
        t[a] = src + hdt * un;
        t[a] -= det * (g.mdiag * pv[a] + g.mfull * sp);
        if (lift) t[a] -= o[a];
    }
    // boundary faces (bit b: the face opposite vertex b): - dt bflux_f |f| / d
    // to each of the face's vertices
    const unsigned bits = pa.ebnd[k];
    if (bits && pa.bflux) {
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            if (!(bits & (1u << b))) continue;
            const double nn = sqrt(n[b][0] * n[b][0] + n[b][1] * n[b][1] + n[b][2] * n[b][2]);
            const double area = (DIM == 2) ? nn : 0.5 * nn;
            const double val = pa.dt * pa.bflux[pa.efc[4 * k + b]] * area / double(DIM);
#pragma unroll
            for (int a = 0; a <= DIM; ++a)
                if (a != b) t[a] -= val;
        }
    }
#pragma unroll
    for (int a = 0; a <= DIM; ++a) contrib[4 * k + a] = t[a];
}

// Pre-projection: element means of the dual-cell fields, (rho K)_k with
// W_u^{n+1,1} = double-tilde W_u, element volume, and c_k = H_k from P^n;
// then the element part of the first Picard iteration's right-hand side.
template <int DIM, bool PER>
__global__ void __launch_bounds__(BLK) k_proj_init(Mesh g, ProjArgs pa, const double *__restrict__ pn,
                                                   double *__restrict__ coef, const double *__restrict__ gd,
                                                   double *__restrict__ contrib)
{
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k >= g.E) return;
    int v[4];
    double ed[3][3], n[4][3];
    elem_corners<DIM, PER>(g, k, v, ed);
    const double det = elem_normals<DIM>(ed, n);
    double rho = 0.0, we = 0.0, wu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        const int f = pa.efc[4 * k + a];
        rho += pa.rho_f[f];
        we += pa.we_f[f];
#pragma unroll
        for (int c = 0; c < DIM; ++c) wu[c] += pa.wu_f[DIM * f + c];
    }
    constexpr double inv = 1.0 / double(DIM + 1);
    rho *= inv;
    we *= inv;
    double ww = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        wu[c] *= inv;
        ww += wu[c] * wu[c];
        pa.ewu[3 * k + c] = wu[c];
    }
    double pv[4];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) pv[a] = pn[v[a]];
    const double rk = ww / (2.0 * rho);
    pa.erho[k] = rho;
    pa.ewe[k] = we;
    pa.erk[k] = rk;
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    pa.evol[k] = det / dfact;
    const double hk = elem_enthalpy<DIM>(pa, k, pv);
    const double wk = (pa.dt * pa.dt * hk) / (dfact * det);
    coef[k] = hk;
    pa.w[k] = wk;
    rhs_elem_write<DIM>(g, pa, k, v, ed, n, det, we, rk, wu, hk, wk, pv, gd, contrib);
}

// Node pass: b_i = the sum of its element contributions, gd_i on a
// Dirichlet node; written in caller order.  Four accumulators take the
// incidences q = 4j + l (fixed pattern, so the sum is reproducible) and keep
// four loads in flight per lane.  Nodes go to XCDs in contiguous chunks, so
// the contributions of shared elements are read through one L2.
__global__ void __launch_bounds__(BLK) k_proj_rhs_node(int N, const int *__restrict__ off, const int *__restrict__ ent,
                                                       const uint8_t *__restrict__ dir, const double *__restrict__ gd,
                                                       const double *__restrict__ contrib,
                                                       const int *__restrict__ new2old, double *__restrict__ b)
{
    const int i = xcd_block(int(blockIdx.x), int(gridDim.x)) * BLK + threadIdx.x;
    if (i >= N) return;
    double bi = 0.0;
    if (dir[i]) {
        bi = gd[i];
    } else {
        const int q0 = off[i], q1 = off[i + 1];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int q = q0;
        for (; q + 4 <= q1; q += 4) {
            int e[4];
#pragma unroll
            for (int l = 0; l < 4; ++l) e[l] = ent[q + l];
#pragma unroll
            for (int l = 0; l < 4; ++l) acc[l] += contrib[e[l]];
        }
        for (int l = 0; q < q1; ++q, ++l) acc[l] += contrib[ent[q]];
        bi = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    b[new2old[i]] = bi;
}

// After a solve: grad(dP) per element, the element momentum W_u - dt grad
// and its (rho K), and c_k = H_k from P^n + dP; with RHS, then the element
// part of the next Picard iteration's right-hand side.
template <int DIM, bool PER, bool RHS>
__global__ void __launch_bounds__(BLK) k_proj_picard(Mesh g, ProjArgs pa, const double *__restrict__ pn,
                                                     const double *__restrict__ dpi, double *__restrict__ coef,
                                                     const double *__restrict__ gd, double *__restrict__ contrib)
{
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k >= g.E) return;
    int v[4];
    double ed[3][3], n[4][3];
    elem_corners<DIM, PER>(g, k, v, ed);
    const double det = elem_normals<DIM>(ed, n);
    double d[4], p0[4], pv[4];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        d[a] = dpi[v[a]];
        p0[a] = pn[v[a]];
        pv[a] = p0[a] + d[a];
    }
    double ww = 0.0, u[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double gc = 0.0;
#pragma unroll
        for (int a = 0; a <= DIM; ++a) gc += d[a] * n[a][c];
        gc /= det;
        pa.egrad[3 * k + c] = gc;
        u[c] = pa.ewu[3 * k + c];
        const double wc = u[c] - pa.dt * gc;
        ww += wc * wc;
    }
    const double rk = ww / (2.0 * pa.erho[k]);
    pa.erk[k] = rk;
    const double hk = elem_enthalpy<DIM>(pa, k, pv);
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    const double wk = (pa.dt * pa.dt * hk) / (dfact * det);
    coef[k] = hk;
    pa.w[k] = wk;
    if constexpr (RHS) rhs_elem_write<DIM>(g, pa, k, v, ed, n, det, pa.ewe[k], rk, u, hk, wk, p0, gd, contrib);
}

// Momentum update on the dual cells: W_u,f - dt (sum_k |T_k| grad_k) / (sum_k |T_k|).
template <int DIM>
__global__ void __launch_bounds__(BLK) k_proj_faces(int F, ProjArgs pa, double *__restrict__ wu_out)
{
    const int f = blockIdx.x * BLK + threadIdx.x;
    if (f >= F) return;
    const int2 ke = pa.fel[f];
    double vs = pa.evol[ke.x], gs[3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) gs[c] = pa.evol[ke.x] * pa.egrad[3 * ke.x + c];
    if (ke.y >= 0) {
        vs += pa.evol[ke.y];
#pragma unroll
        for (int c = 0; c < DIM; ++c) gs[c] += pa.evol[ke.y] * pa.egrad[3 * ke.y + c];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) wu_out[DIM * f + c] = pa.wu_f[DIM * f + c] - pa.dt * (gs[c] / vs);
}

// gd_i = P^{n+1}_B - P^n_B on Dirichlet nodes (pb null: 0), 0 elsewhere.
__global__ void __launch_bounds__(BLK) k_proj_lift(int N, const int *__restrict__ new2old,
                                                   const uint8_t *__restrict__ dir, const double *__restrict__ pb,
                                                   const double *__restrict__ pn, double *__restrict__ gd)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i >= N) return;
    gd[i] = (dir[i] && pb) ? pb[new2old[i]] - pn[i] : 0.0;
}

// out = a + b (caller order)
__global__ void __launch_bounds__(BLK) k_add(int N, const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ out)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i < N) out[i] = a[i] + b[i];
}

// out[perm[k]] = v[k]
__global__ void __launch_bounds__(BLK) k_scatter_elem(int E, const int *__restrict__ perm,
                                                      const double *__restrict__ v, double *__restrict__ out)
{
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k < E) out[perm[k]] = v[k];
}

// Post-projection (Sec. 3.5, eq. WEupdatek): the total energy per primal
// element from the intermediate energy and the enthalpy flux through its
// faces, then back to the dual cells.  On primal face l of T_k the momentum
// is W_u^{n+1} of the dual cell of l and the enthalpy H_l = g1 P_l / rho_l,
// P_l the mean of the face's vertex pressures P^{n+1}; the outward area
// vector of face l is -n_l / (d-1)!.
template <int DIM, bool PER>
__global__ void __launch_bounds__(BLK) k_post_elem(Mesh g, ProjArgs pa, const double *__restrict__ pnew,
                                                   double *__restrict__ ewe_new)
{
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k >= g.E) return;
    int v[4];
    double ed[3][3], n[4][3];
    elem_corners<DIM, PER>(g, k, v, ed);
    const double det = elem_normals<DIM>(ed, n);
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    constexpr double ffact = (DIM == 2) ? 1.0 : 2.0;   // (d-1)!
    double pv[4];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) pv[a] = pnew[v[a]];
    double we = 0.0, flux = 0.0;
#pragma unroll
    for (int l = 0; l <= DIM; ++l) {
        const int f = pa.efc[4 * k + l];
        we += pa.we_f[f];
        double pf = 0.0;
#pragma unroll
        for (int b = 0; b <= DIM; ++b)
            if (b != l) pf += pv[b];
        const double hl = pa.g1 * (pf / double(DIM)) / pa.rho_f[f];
        double wn = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) wn += pa.wu_f[DIM * f + c] * n[l][c];
        flux -= hl * wn / ffact;
    }
    const double vol = det / dfact;
    pa.evol[k] = vol;
    ewe_new[k] = we / double(DIM + 1) - pa.dt * flux / vol;
}

// W_E,f = sum_k |T_kf| W_E,k / |C_f| over the one or two elements of f.
__global__ void __launch_bounds__(BLK) k_post_faces(int F, ProjArgs pa, const double *__restrict__ ewe_new,
                                                    double *__restrict__ we_out)
{
    const int f = blockIdx.x * BLK + threadIdx.x;
    if (f >= F) return;
    const int2 ke = pa.fel[f];
    double vs = pa.evol[ke.x], es = pa.evol[ke.x] * ewe_new[ke.x];
    if (ke.y >= 0) {
        vs += pa.evol[ke.y];
        es += pa.evol[ke.y] * ewe_new[ke.y];
    }
    we_out[f] = es / vs;
}

// -------------------------------------------------------- transport stage
// First-order explicit finite volumes on the dual cells (Sec. 3.2, eq.
// discrf_mass / discrf_momentum / discrf_energy) with the modified Rusanov
// flux of eq. flux.  Inside element k the dual cells of faces a and b meet
// on the triangle (3D) or segment (2D) that joins the barycenter to the
// primal edge (vertex) they share; its area vector from cell a to cell b is
// eta_ab = |T| d/(d+1) (grad phi_a - grad phi_b) = d/((d+1) d!) (n_a - n_b).

struct TransArgs {
    const int4 *trec;             // 2 per (face, side): vertex ids, then faces opposite them (-1: no element)
    const double *rho, *wu, *we;  // per face; wu: dim per face
    const int2 *fsl;              // per face: element slots 4k + a of its two sides (-1: none)
    const double *grad;           // LADER: Galerkin gradients of rho and W_u per element (DIM + DIM^2 each)
    const int *oslot;             // LADER: per element slot 4k + a, the other slot of face a's cell (-1: none)
    double calpha;                // artificial viscosity coefficient c_alpha
    double mu;                    // dynamic viscosity (0: inviscid)
    double lam_r;                 // thermal conductivity over the gas constant, lambda / R
    double dt;
    double g[3];                  // gravity
};

// One cell's state for the flux: rho, 1/rho, W_u and rho K = |W_u|^2 / (2 rho),
// formed once per state by the same expressions in every lane.
struct CellState {
    double r, ir, k;
};

__device__ __forceinline__ CellState cell_state(double r, const double u[3])
{
    const double ir = 1.0 / r;
    const double w = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return {r, ir, 0.5 * w * ir};
}

// Rusanov flux from the cell with state (si, ui) to the cell with (sj, uj)
// across eta: acc += phi.  Swapping the cells and negating eta gives -phi
// bit for bit (each step is symmetric or changes sign exactly, and a state's
// 1/rho and rho K do not depend on the side it is on), so the two cells of
// a dual face see opposite fluxes.
__device__ __forceinline__ void rusanov_add(const CellState &si, const double ui[3], const CellState &sj,
                                            const double uj[3], const double eta[3], double calpha, double acc[5])
{
    const double ri = si.r, rj = sj.r, ki = si.k, kj = sj.k;
    double a = 0.0, b = 0.0, en = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a += ui[c] * eta[c];
        b += uj[c] * eta[c];
        en += eta[c] * eta[c];
    }
    const double vi = a * si.ir, vj = b * sj.ir;     // U . eta
    const double ars = fmax(fabs(vi), fabs(vj)) + ((calpha > 0.0) ? calpha * sqrt(en) : 0.0);
    acc[0] += 0.5 * (a + b) - 0.5 * ars * (rj - ri);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[1 + c] += 0.5 * (ui[c] * vi + uj[c] * vj) - 0.5 * ars * (uj[c] - ui[c]);
    acc[4] += 0.5 * (ki * vi + kj * vj) - 0.5 * ars * (kj - ki);
}

// Per (face f, side s) the element of f on that side as two records: its
// vertex ids (internal order, Dirichlet bit cleared) and the faces opposite
// them, f itself at its local index; -1 in the second record when f has no
// element on that side.  Lane 2f + s of the transport kernel reads its two
// records with one coalesced load each, in place of a slot, connectivity
// and face lookup that depend on one another.
__global__ void __launch_bounds__(BLK) k_tr_records(int F, const int2 *__restrict__ fsl,
                                                    const int4 *__restrict__ conn, const int *__restrict__ efc,
                                                    int4 *__restrict__ trec)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    if (t >= 2 * F) return;
    const int2 sl = fsl[t >> 1];
    const int slot = (t & 1) ? sl.y : sl.x;
    int4 va = make_int4(0, 0, 0, 0), fa = make_int4(-1, -1, -1, -1);
    if (slot >= 0) {
        const int k = slot >> 2;
        const int4 c = conn[k];
        va = make_int4(c.x & 0x7fffffff, c.y & 0x7fffffff, c.z & 0x7fffffff, c.w & 0x7fffffff);
        fa = make_int4(efc[4 * k], efc[4 * k + 1], efc[4 * k + 2], efc[4 * k + 3]);
    }
    trec[2 * t] = va;
    trec[2 * t + 1] = fa;
}

// Per element slot s = 4k + a (a <= d): the other slot of the cell of k's
// face a, whose element is that cell's upwind element for this side (-1 on
// the boundary).  Built once, so that the LADER element pass reaches the
// upwind gradient without looking up the face first.
__global__ void __launch_bounds__(BLK) k_tr_oslot(int n_slots, int nv, const int *__restrict__ efc,
                                                  const int2 *__restrict__ fsl, int *__restrict__ oslot)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= n_slots) return;
    int o = -1;
    if ((s & 3) < nv) {
        const int2 sl = fsl[efc[s]];
        o = (sl.x == s) ? sl.y : sl.x;
    }
    oslot[s] = o;
}

// LADER (Sec. 3.2.1), the gradients: on every primal element the Galerkin
// (Crouzeix-Raviart) gradient of rho and of each momentum component from the
// states of its d+1 dual cells, whose face-based basis functions are
// 1 - d phi_a: grad W = -d sum_a W_a grad phi_a = -(d / det) sum_a W_a n_a.
// Per element (internal order) DIM + DIM^2 doubles: grad rho, then
// grad W_u,c for c = 0 .. DIM-1.
template <int DIM, bool PER>
__global__ void __launch_bounds__(BLK) k_tr_grad(Mesh g, const int *__restrict__ efc, const double *__restrict__ rho,
                                                 const double *__restrict__ wu, double *__restrict__ grad)
{
    constexpr int NG = DIM + DIM * DIM;
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k >= g.E) return;
    int v[4];
    double ed[3][3], n[4][3];
    elem_corners<DIM, PER>(g, k, v, ed);
    const double det = elem_normals<DIM>(ed, n);
    double gr[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) gr[j] = 0.0;
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        const int f = efc[4 * k + a];
        const double r = rho[f];
#pragma unroll
        for (int e = 0; e < DIM; ++e) gr[e] += r * n[a][e];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double w = wu[DIM * f + c];
#pragma unroll
            for (int e = 0; e < DIM; ++e) gr[DIM + c * DIM + e] += w * n[a][e];
        }
    }
    const double sc = -double(DIM) / det;
#pragma unroll
    for (int j = 0; j < NG; ++j) grad[int64_t(NG) * k + j] = gr[j] * sc;
}

// LADER Steps 1-3 for one side of a dual face: the cell's state (r, u), the
// gradients of the centred element gc and of the cell's other (upwind)
// element gu (gc again when there is none), dl = N_ij - N_i.  Per scalar
// (rho, then each momentum component) the ENO choice takes the upwind
// gradient when its extrapolation is not larger in magnitude; the
// extrapolated state is evolved by half a time step (hdt = dt/2) with the
// Cauchy-Kovalevskaya form of the mass and momentum equations written with
// the chosen gradients: d rho/dt = -div W_u, d W_u/dt = -div(W_u (x) U)
// - grad P + rho g, div(W_u (x) U) = (grad W_u) U + W_u div U,
// div U = (div W_u - U . grad rho) / rho.  Both lanes that see the face
// evaluate this with the same inputs in the same order.
template <int DIM>
__device__ __forceinline__ void lader_side(double r, const double u[3], const double *__restrict__ gc,
                                           const double *__restrict__ gu, const double dl[3], const double gp[3],
                                           const double gv[3], double hdt, double &rbar, double ubar[3])
{
    double G[1 + DIM][DIM], w[1 + DIM];
#pragma unroll
    for (int sc = 0; sc <= DIM; ++sc) {
        const int o = (sc == 0) ? 0 : DIM + (sc - 1) * DIM;
        double dc = 0.0, du = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            dc += gc[o + e] * dl[e];
            du += gu[o + e] * dl[e];
        }
        const bool up = fabs(du) <= fabs(dc);
#pragma unroll
        for (int e = 0; e < DIM; ++e) G[sc][e] = up ? gu[o + e] : gc[o + e];
        w[sc] = ((sc == 0) ? r : u[sc - 1]) + (up ? du : dc);
    }
    const double ir = 1.0 / w[0];
    double U[DIM], tr = 0.0, ug = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        U[c] = w[1 + c] * ir;
        tr += G[1 + c][c];
    }
#pragma unroll
    for (int e = 0; e < DIM; ++e) ug += U[e] * G[0][e];
    const double divu = (tr - ug) * ir;
    rbar = w[0] - hdt * tr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c < DIM) {
            double t = 0.0;
#pragma unroll
            for (int e = 0; e < DIM; ++e) t += G[1 + c][e] * U[e];
            ubar[c] = w[1 + c] - hdt * (t + w[1 + c] * divu + gp[c] - w[0] * gv[c]);
        } else {
            ubar[c] = 0.0;
        }
    }
}

// The diffusive terms of cell a's side on element T_k (first order in
// time): the viscous stress from the Crouzeix-Raviart gradient of the face
// velocities, and the heat flux from the cells' temperatures.  rs, us: the
// states of T_k's d+1 faces; n, det: its adjugate normals and determinant;
// pn, v: the vertex pressures.
template <int DIM>
__device__ __forceinline__ void visc_side(int a, const double rs[4], const double us[4][3], const double n[4][3],
                                          double det, const double *__restrict__ pn, const int v[4],
                                          const TransArgs &ta, double acc[5])
{
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    constexpr double ceta = double(DIM) / (double(DIM + 1) * dfact);
    // Crouzeix-Raviart gradient of the face velocities on T_k,
    // grad u = -d sum_b u_b (x) grad phi_b, and the stress
    // tau = mu (grad u + grad u^T - 2/3 div u I), constant on T_k
    double vel[4][DIM], gu[DIM][DIM], tau[DIM][DIM], ir[4];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        ir[b] = 1.0 / rs[b];
#pragma unroll
        for (int c = 0; c < DIM; ++c) vel[b][c] = us[b][c] * ir[b];
    }
    const double gs = -double(DIM) / det;
    double dv = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b <= DIM; ++b) t += vel[b][c] * n[b][e];
            gu[c][e] = t * gs;
            if (c == e) dv += gu[c][e];
        }
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int e = 0; e < DIM; ++e)
            tau[c][e] = ta.mu * (gu[c][e] + gu[e][c] - ((c == e) ? (2.0 / 3.0) * dv : 0.0));
    // momentum: minus the integral of tau eta over the cell's dual
    // faces in T_k, which close on n_a / (d-1)!
    constexpr double ffact = (DIM == 2) ? 1.0 : 2.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) t += tau[c][e] * n[a][e];
        acc[1 + c] -= t / ffact;
    }
    // energy: minus (tau u) . eta on each dual face, u the mean
    // velocity of the two cells
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        if (b == a) continue;
        double te = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            double t = 0.0;
#pragma unroll
            for (int e = 0; e < DIM; ++e) t += tau[c][e] * (ceta * (n[a][e] - n[b][e]));
            te += t * (0.5 * (vel[a][c] + vel[b][c]));
        }
        acc[4] -= te;
    }
    // heat flux Q = -lambda grad Theta with Theta = P / (rho R) on
    // each cell, P the mean of its face's vertex pressures, and
    // the same Galerkin gradient; Q . eta over the cell's dual
    // faces in T_k closes on Q . n_a / (d-1)!
    double pv[4], ps = 0.0;
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        pv[b] = pn[v[b]];
        ps += pv[b];
    }
    double qn = 0.0;
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        const double th = (ps - pv[b]) * (1.0 / double(DIM)) * ir[b];
        double nn = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) nn += n[b][e] * n[a][e];
        qn += th * nn;
    }
    acc[4] -= ta.lam_r * gs * qn / ffact;
}

// One pass per dual cell f, two lanes per cell (adjacent lanes 2f and
// 2f+1 of a wave): lane `side` takes the cell's element in that slot, the
// fluxes to the element's other d faces (ascending local index) and its
// share |T|/(d+1) grad(P^n) of the pressure force; the even lane adds the
// odd lane's sums to its own (side 0 + side 1) and writes the update with
// the gravity sources.  VISC adds the diffusive terms: the viscous stress
// and the heat flux.  Cells go to XCDs in contiguous chunks (xcd_block):
// the element and neighbour data of nearby cells then share one L2, which
// more than halves the kernel's HBM reads.
template <int DIM, bool PER, bool VISC>
__global__ void __launch_bounds__(BLK) k_tr_cell(Mesh g, TransArgs ta, const double *__restrict__ pn, int F,
                                                 double *__restrict__ rho_out, double *__restrict__ wu_out,
                                                 double *__restrict__ we_out)
{
    const int t = xcd_block(int(blockIdx.x), int(gridDim.x)) * BLK + threadIdx.x;
    const int f = t >> 1, side = t & 1;
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    constexpr double ceta = double(DIM) / (double(DIM + 1) * dfact);
    constexpr double share = 1.0 / (dfact * double(DIM + 1));
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double vol = 0.0, r0 = 1.0, u0[3] = {0.0, 0.0, 0.0};
    const bool live = f < F;
    if (live) {
        r0 = ta.rho[f];
#pragma unroll
        for (int c = 0; c < DIM; ++c) u0[c] = ta.wu[DIM * f + c];
        const int4 ra = ta.trec[2 * t], rb = ta.trec[2 * t + 1];
        if (rb.x >= 0) {
            const int v[4] = {ra.x, ra.y, ra.z, ra.w};
            const int fe4[4] = {rb.x, rb.y, rb.z, rb.w};    // fe4[a] == f
            const int a = (rb.y == f) ? 1 : (rb.z == f) ? 2 : (DIM == 3 && rb.w == f) ? 3 : 0;
            double ed[3][3], n[4][3];
            elem_corners_of<DIM, PER>(g, v, ed);
            const double det = elem_normals<DIM>(ed, n);
            vol = det * share;
            // states of the element's faces (the cell's own at a); the
            // viscous stress needs all of them at once
            double rs[4], us[4][3];
            const CellState s0 = cell_state(r0, u0);
            if constexpr (VISC) {
#pragma unroll
                for (int b = 0; b <= DIM; ++b) {
                    const int fb = fe4[b];
                    rs[b] = (b == a) ? r0 : ta.rho[fb];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        us[b][c] = (b == a) ? u0[c] : ((c < DIM) ? ta.wu[DIM * fb + c] : 0.0);
                }
            }
#pragma unroll
            for (int b = 0; b <= DIM; ++b) {
                if (b == a) continue;
                double eta[3], rb, ub[3];
                if constexpr (VISC) {
                    rb = rs[b];
#pragma unroll
                    for (int c = 0; c < 3; ++c) ub[c] = us[b][c];
                } else {
                    const int fb = fe4[b];
                    rb = ta.rho[fb];
#pragma unroll
                    for (int c = 0; c < 3; ++c) ub[c] = (c < DIM) ? ta.wu[DIM * fb + c] : 0.0;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) eta[c] = ceta * (n[a][c] - n[b][c]);
                rusanov_add(s0, u0, cell_state(rb, ub), ub, eta, ta.calpha, acc);
            }
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                double tp = 0.0;
#pragma unroll
                for (int b = 0; b <= DIM; ++b) tp += pn[v[b]] * n[b][c];
                acc[1 + c] += tp * share;
            }
            if constexpr (VISC) visc_side<DIM>(a, rs, us, n, det, pn, v, ta, acc);
        }
    }
    // the pair's lanes are 2f and 2f+1 of the same wave (BLK is a multiple of 64)
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += __shfl_xor(acc[c], 1);
    vol += __shfl_xor(vol, 1);
    if (!live || side) return;
    const double q = ta.dt / vol;   // dt / |C_f|
    rho_out[f] = r0 - q * acc[0];
    double gw = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        gw += ta.g[c] * u0[c];
        wu_out[DIM * f + c] = u0[c] - q * acc[1 + c] + ta.dt * r0 * ta.g[c];
    }
    we_out[f] = ta.we[f] - q * acc[4] + ta.dt * gw;
}

// LADER (Sec. 3.2.1), the element pass: four adjacent lanes per element k
// (lanes 4k' .. 4k'+3 of a wave; in 2D the fourth idles), lane a for the
// side of k's face a, that is of the dual cell f_a.  Lane a forms, for each
// other face b (ascending), the evolved state of its cell at the dual face
// between f_a and f_b (lader_side with the centred gradient of k and the
// upwind gradient of f_a's other element); the state of f_b's side at the
// same dual face is lane b's, read from LDS.  So each side of
// each dual face is evolved once, and the two lanes of a dual face see the
// same two states and opposite fluxes.  The lane sums its Rusanov fluxes in
// ascending b, adds its share of the pressure force (and with VISC the
// diffusive terms) and writes them with the share |T|/(d+1) of the cell
// volume as the slot record of (k, a): 6 doubles at 6 (4k + a).
template <int DIM, bool PER, bool VISC>
__global__ void __launch_bounds__(BLK) k_lader_elem(Mesh g, TransArgs ta, const int *__restrict__ efc,
                                                    const double *__restrict__ pn, double *__restrict__ slots)
{
    constexpr int NG = DIM + DIM * DIM, NV = DIM + 1;
    constexpr double dfact = (DIM == 2) ? 2.0 : 6.0;
    constexpr double ceta = double(DIM) / (double(DIM + 1) * dfact);
    constexpr double share = 1.0 / (dfact * double(DIM + 1));
    const int t = xcd_block(int(blockIdx.x), int(gridDim.x)) * BLK + threadIdx.x;
    const int k = t >> 2, a = t & 3;
    const bool live = k < g.E && a < NV;
    const int kk = (k < g.E) ? k : g.E - 1;   // lanes past the end mirror the last element
    int v[4];
    double ed[3][3], n[4][3];
    elem_corners<DIM, PER>(g, kk, v, ed);
    const double det = elem_normals<DIM>(ed, n);
    // vertex positions relative to vertex 0, barycentre, grad P^n on k
    // (divisions by d + 1, d and det as products with reciprocals)
    double X[4][3], Bc[3], gp[3], tp[3];
    const double idet = 1.0 / det;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        X[0][c] = 0.0;
        double s = 0.0, sp = 0.0;
#pragma unroll
        for (int b = 1; b <= DIM; ++b) {
            X[b][c] = ed[b - 1][c];
            s += X[b][c];
        }
#pragma unroll
        for (int b = 0; b <= DIM; ++b) sp += pn[v[b]] * n[b][c];
        Bc[c] = s * (1.0 / double(DIM + 1));
        gp[c] = (c < DIM) ? sp * idet : 0.0;
        tp[c] = sp;
    }
    // this lane's cell, its state and its upwind element (the other
    // element of face a; k itself on the boundary)
    const int al = (a < NV) ? a : 0;
    const int fa = efc[4 * kk + al];
    const double r0 = ta.rho[fa];
    double u0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u0[c] = (c < DIM) ? ta.wu[DIM * fa + c] : 0.0;
    const int so = ta.oslot[4 * kk + al];
    const double *gk = ta.grad + int64_t(NG) * kk;
    const double *ga = (so < 0) ? gk : ta.grad + int64_t(NG) * (so >> 2);
    const double hdt = 0.5 * ta.dt;
    // the lane's normal n_a, and per partner j (b = j or j + 1, ascending)
    // the partner's normal and position, chosen without indexing local
    // arrays by the lane number
    double na[3], nb[3][3], Xb[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        na[c] = n[0][c];
#pragma unroll
        for (int q = 1; q <= DIM; ++q)
            if (al == q) na[c] = n[q][c];
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            const bool sh = j >= al;
            nb[j][c] = sh ? n[j + 1][c] : n[j][c];
            Xb[j][c] = sh ? X[j + 1][c] : X[j][c];
        }
    }
    // evolved states of this side at its d dual faces (partner b ascending)
    // go to LDS, (lane, j)-major, 4 doubles each: the lanes of a dual face
    // read each other's there
    __shared__ double sE[BLK * DIM * 4];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        double dl[3], er, eu[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) dl[c] = (Bc[c] - Xb[j][c]) * (1.0 / double(DIM));
        lader_side<DIM>(r0, u0, gk, ga, dl, gp, ta.g, hdt, er, eu);
        double *e = sE + 4 * (DIM * int(threadIdx.x) + j);
        e[0] = er;
        e[1] = eu[0];
        e[2] = eu[1];
        e[3] = eu[2];
    }
    __syncthreads();
    if (!live) return;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        const int b = j + ((j >= al) ? 1 : 0);
        const int jb = al - ((al > b) ? 1 : 0);   // this lane's index among lane b's partners
        const double *e = sE + 4 * (DIM * int(threadIdx.x) + j);
        const double *fp = sE + 4 * (DIM * int((threadIdx.x & ~3u) + unsigned(b)) + jb);
        const double eu[3] = {e[1], e[2], e[3]}, fu[3] = {fp[1], fp[2], fp[3]};
        double eta[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) eta[c] = ceta * (na[c] - nb[j][c]);
        rusanov_add(cell_state(e[0], eu), eu, cell_state(fp[0], fu), fu, eta, ta.calpha, acc);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[1 + c] += tp[c] * share;
    if constexpr (VISC) {
        double rs[4], us[4][3];
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            const int fb = efc[4 * kk + b];
            rs[b] = (b == al) ? r0 : ta.rho[fb];
#pragma unroll
            for (int c = 0; c < 3; ++c) us[b][c] = (b == al) ? u0[c] : ((c < DIM) ? ta.wu[DIM * fb + c] : 0.0);
        }
        visc_side<DIM>(al, rs, us, n, det, pn, v, ta, acc);
    }
    double *out = slots + 6 * (int64_t(4) * k + a);
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = acc[c];
    out[5] = det * share;
}

// LADER, the cell pass: cell f adds the slot records of its two sides
// (side 0 + side 1) and takes the update with the gravity sources, as the
// first-order kernel does.
template <int DIM>
__global__ void __launch_bounds__(BLK) k_lader_cell(TransArgs ta, int F, const double *__restrict__ slots,
                                                    double *__restrict__ rho_out, double *__restrict__ wu_out,
                                                    double *__restrict__ we_out)
{
    const int f = xcd_block(int(blockIdx.x), int(gridDim.x)) * BLK + threadIdx.x;
    if (f >= F) return;
    const int2 sl = ta.fsl[f];
    double acc[6];
    const double *r0p = slots + 6 * int64_t(sl.x);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = r0p[c];
    if (sl.y >= 0) {
        const double *r1p = slots + 6 * int64_t(sl.y);
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += r1p[c];
    }
    const double r0 = ta.rho[f];
    double u0[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) u0[c] = ta.wu[DIM * f + c];
    const double q = ta.dt / acc[5];   // dt / |C_f|
    rho_out[f] = r0 - q * acc[0];
    double gw = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        gw += ta.g[c] * u0[c];
        wu_out[DIM * f + c] = u0[c] - q * acc[1 + c] + ta.dt * r0 * ta.g[c];
    }
    we_out[f] = ta.we[f] - q * acc[4] + ta.dt * gw;
}

// ----------------------------------------------------------- batched solve
// Many meshes advance their CG iterations together: one launch runs the
// apply of iteration k for every (mesh, slot) pair, the next the update.  The
// iteration number lives in device memory (each kernel reads the field the
// previous kernel wrote and writes the other one), so a sequence of
// iterations can be captured once in a HIP graph and replayed.  Meshes that
// have converged skip their slots.

template <class R>
struct BatchMeshT {
    int dim, N;
    MeshT<R> g;
    TileArgsT<R> ta;
    R *x, *r, *q, *p0, *p1;   // FP32 batches: the inner solve's d, r, q, p
    double *hist;
    CGState *st;
    double *part_pq, *rr0, *rr1;
    int n_ab, n_vb;   // apply / update virtual blocks of this mesh
};
using BatchMesh = BatchMeshT<double>;

struct BatchCtl {
    int k_apply;   // iteration the next apply launch runs
    int k_update;  // iteration the next update launch runs
    int n_done;
    int failed;    // persistent launches: a grid barrier timed out
};

// Grid barrier state of the persistent launches (zero at creation; every
// launch leaves it as it found it but for the generations).
// Each counter has a 128-byte line of its own, so that the blocks polling
// one XCD's generation do not contend with the arrivals of another.
constexpr int MAX_XCC = 16;
struct alignas(128) BarWord {
    unsigned v;
    unsigned pad[31];
};
struct GridBar {
    BarWord reg[MAX_XCC];   // blocks of the current launch per XCD (registration)
    BarWord cnt[MAX_XCC];   // arrivals per XCD at the current barrier
    BarWord gen[MAX_XCC];   // barrier generation per XCD
    BarWord n_reg;          // blocks registered in the current launch
    BarWord gcnt, ggen;     // XCD leaders' arrivals and generation
};

// The apply of iteration k (launch index) for one (mesh, tile slot) pair
// ms.  Each solve numbers its iterations from its first launch (k_first)
// and picks its p and r.r buffers by the parity of that number, as a
// single-mesh solve does; so a solve may start, or continue, at any launch.
// C: size class (128-node tiles) covering every mesh of the batch.
template <int C, class R, bool PER>
__device__ __forceinline__ void batch_apply_slot(const BatchMeshT<R> *__restrict__ meshes, int2 ms, int k, R *smem,
                                                 double *red)
{
    const BatchMeshT<R> &M = meshes[ms.x];
    const int kl = k - M.st->k_first + 1;
    IterT<R> it;
    it.k = kl;
    it.first = (kl == 1) ? 1 : 0;
    it.r = M.r;
    it.p_old = (kl & 1) ? M.p0 : M.p1;   // p_{k-1}
    it.p_new = (kl & 1) ? M.p1 : M.p0;   // p_k
    it.q = M.q;
    it.st = M.st;
    it.hist = M.hist;
    it.part_pq = M.part_pq;
    it.rr_cur = (kl & 1) ? M.rr0 : M.rr1;
    it.rr_prev = (kl & 1) ? M.rr1 : M.rr0;
    it.n_vblocks = M.n_vb;
    constexpr TileClass tc = TILE_CLASSES[C];
    static_assert(tc.t == 128, "batched meshes use 128-node tiles");
    if (M.dim == 3)
        apply_tiled_body<3, true, R, 128, tc.ipt, tc.lm, BLK, PER>(M.g, M.ta, nullptr, M.q, it, smem, red, ms.y,
                                                                  M.n_ab);
    else
        apply_tiled_body<2, true, R, 128, tc.ipt, tc.lm, BLK, PER>(M.g, M.ta, nullptr, M.q, it, smem, red, ms.y,
                                                                  M.n_ab);
}

// The vector update of iteration k for one (mesh, node slot) pair ms.
template <class R>
__device__ __forceinline__ void batch_update_slot(const BatchMeshT<R> *__restrict__ meshes, int2 ms, int k,
                                                  double *red)
{
    const BatchMeshT<R> &M = meshes[ms.x];
    const int kl = k - M.st->k_first + 1;
    update_body<R>(M.N, M.x, M.r, (kl & 1) ? M.p1 : M.p0, M.q, M.st, M.part_pq, M.n_ab,
                   (kl & 1) ? M.rr0 : M.rr1, (kl & 1) ? M.rr1 : M.rr0, red, ms.y, M.n_vb);
}

// Two launches per iteration: the apply over the slot table, then the
// update.  The iteration number lives in ctl (each kernel reads the field
// the previous one wrote and writes the other), so a chunk of iterations
// can be captured in a HIP graph and replayed.
template <int C, class R, bool PER>
__global__ void __launch_bounds__(BLK, (tile_waves<R, TILE_CLASSES[C].t, TILE_CLASSES[C].lm>())) k_batch_apply(const BatchMeshT<R> *__restrict__ meshes,
                                                     const int2 *__restrict__ slots, BatchCtl *ctl)
{
    extern __shared__ double smem_d[];
    __shared__ double red[BLK / 64];
    const int k = ctl->k_apply;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->k_update = k;
    batch_apply_slot<C, R, PER>(meshes, slots[blockIdx.x], k, reinterpret_cast<R *>(smem_d), red);
}

template <class R>
__global__ void __launch_bounds__(BLK) k_batch_update(const BatchMeshT<R> *__restrict__ meshes,
                                                      const int2 *__restrict__ slots, BatchCtl *ctl)
{
    __shared__ double red[BLK / 64];
    const int k = ctl->k_update;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->k_apply = k + 1;
    batch_update_slot<R>(meshes, slots[blockIdx.x], k, red);
}

// Grid barrier of a persistent launch (every block resident: cooperative
// launch), two-level so that each XCD's L2 is written back once per
// barrier, not once per block.  Blocks on one XCD share its L2: a block
// makes its stores reach that L2 (every wave waits for its stores), and
// thread 0 arrives on the XCD's counter.  The last block of the XCD to
// arrive is its leader: it releases at agent scope (writing back the L2,
// which now holds every store of the XCD's blocks), arrives on the global
// counter of leaders, waits for the leaders' generation to move, acquires
// at agent scope and only then advances the XCD's generation; the other
// blocks of the XCD wait for that and acquire at agent scope themselves (an
// invalidate of the L1 alone was measured to leave stale lines visible).
// Waits poll with relaxed loads and are bounded by
// wall-clock time (the 100 MHz constant clock, `limit` ticks): a block that
// waits longer marks the launch failed and returns false, as does every
// block once the mark is set, so a launch ends in bounded time whatever
// happens to its blocks.
__device__ __forceinline__ unsigned xcc_id()
{
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & unsigned(MAX_XCC - 1);
}

// Wait (thread 0) until *w differs from v; false on time-out or failure mark.
__device__ __forceinline__ bool bar_wait(const unsigned *w, unsigned v, BatchCtl *ctl, long long limit)
{
    const long long t0 = wall_clock64();
    // the clock and the shared failure mark are looked at every 32nd poll
    for (unsigned n = 1; __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == v; ++n) {
        if ((n & 31u) == 0u && (wall_clock64() - t0 > limit ||
                                __hip_atomic_load(&ctl->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(&ctl->failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

struct BarLane {
    unsigned xcc, n_xcc, n_groups;   // this block's XCD, blocks on it, XCDs with blocks
};

// Registration at the start of a launch: every block counts itself on its
// XCD; once all have, each learns its XCD's block count and the number of
// XCDs in use.  Thread 0's view is broadcast through ok_lds / bl_lds.
__device__ bool bar_register(GridBar *gb, BatchCtl *ctl, long long limit, BarLane *bl_lds, int *ok_lds)
{
    if (threadIdx.x == 0) {
        const unsigned x = xcc_id();
        __hip_atomic_fetch_add(&gb->reg[x].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned done = __hip_atomic_fetch_add(&gb->n_reg.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        bool ok = true;
        if (done < gridDim.x) {
            const long long t0 = wall_clock64();
            for (unsigned n = 1; __hip_atomic_load(&gb->n_reg.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x;
                 ++n) {
                if ((n & 31u) == 0u &&
                    (wall_clock64() - t0 > limit ||
                     __hip_atomic_load(&ctl->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                    __hip_atomic_store(&ctl->failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        unsigned groups = 0;
        for (int k = 0; k < MAX_XCC; ++k)
            groups += (__hip_atomic_load(&gb->reg[k].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ? 1u : 0u;
        bl_lds->xcc = x;
        bl_lds->n_xcc = __hip_atomic_load(&gb->reg[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bl_lds->n_groups = groups;
        *ok_lds = ok ? 1 : 0;
    }
    __syncthreads();
    return *ok_lds != 0;
}

__device__ bool grid_barrier(GridBar *gb, BatchCtl *ctl, const BarLane &bl, long long limit, int *ok_lds)
{
    // this wave's stores reach the L2 before thread 0 arrives
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        const unsigned x = bl.xcc;
        const unsigned g = __hip_atomic_load(&gb->gen[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(&gb->cnt[x].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == bl.n_xcc) {
            __hip_atomic_store(&gb->cnt[x].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned gg = __hip_atomic_load(&gb->ggen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned a2 = __hip_atomic_fetch_add(&gb->gcnt.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (a2 == bl.n_groups) {
                __hip_atomic_store(&gb->gcnt.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&gb->ggen.v, gg + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = bar_wait(&gb->ggen.v, gg, ctl, limit);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&gb->gen[x].v, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = bar_wait(&gb->gen[x].v, g, ctl, limit);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (__hip_atomic_load(&ctl->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = false;
        *ok_lds = ok ? 1 : 0;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// Persistent batched CG: one cooperative launch of as many blocks as can be
// resident runs `count` iterations over the slot tables; in each, the
// blocks stride over the apply slots, meet at a grid barrier, stride over
// the update slots and meet again.  The per-slot work is that of
// k_batch_apply / k_batch_update, so results equal theirs bit for bit.
template <int C, class R, bool PER>
__global__ void __launch_bounds__(BLK, (tile_waves<R, TILE_CLASSES[C].t, TILE_CLASSES[C].lm>())) k_batch_persistent(const BatchMeshT<R> *__restrict__ meshes,
                                                          const int2 *__restrict__ aslots, int na,
                                                          const int2 *__restrict__ uslots, int nu, BatchCtl *ctl,
                                                          GridBar *gb, int count, long long limit)
{
    extern __shared__ double smem_d[];
    __shared__ double red[BLK / 64];
    __shared__ int ok_lds;
    __shared__ BarLane bl_lds;
    R *smem = reinterpret_cast<R *>(smem_d);
    // every block reads the first iteration before the first barrier; block
    // 0 writes the next one after the last
    const int k0 = ctl->k_apply;
    bool ok = bar_register(gb, ctl, limit, &bl_lds, &ok_lds);
    const BarLane bl = bl_lds;
    for (int i = 0; i < count && ok; ++i) {
        for (int j = blockIdx.x; j < na; j += gridDim.x) {
            batch_apply_slot<C, R, PER>(meshes, aslots[j], k0 + i, smem, red);
            __syncthreads();
        }
        ok = grid_barrier(gb, ctl, bl, limit, &ok_lds);
        if (!ok) break;
        for (int j = blockIdx.x; j < nu; j += gridDim.x) {
            batch_update_slot<R>(meshes, uslots[j], k0 + i, red);
            __syncthreads();
        }
        ok = grid_barrier(gb, ctl, bl, limit, &ok_lds);
    }
    // after the last barrier every block has read its registration: block 0
    // clears it for the next launch
    if (ok && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < MAX_XCC; ++k) __hip_atomic_store(&gb->reg[k].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&gb->n_reg.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ctl->k_update = k0 + count - 1;
        ctl->k_apply = k0 + count;
    }
}

__global__ void k_set_done(CGState *st)
{
    if (threadIdx.x == 0) st->done = 1;
}

// One block: number of finished meshes, and a copy of every state.
template <class R>
__global__ void __launch_bounds__(BLK) k_batch_status(const BatchMeshT<R> *__restrict__ meshes, int n, BatchCtl *ctl,
                                                      CGState *states)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int c = 0;
    for (int m = threadIdx.x; m < n; m += BLK) {
        const CGState s = *meshes[m].st;
        states[m] = s;
        c += s.done ? 1 : 0;
    }
    atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) ctl->n_done = cnt;
}

// Mixed precision: r32 = r (rounded), d32 = 0, partials of r32.r32 (FP64).
__global__ void __launch_bounds__(BLK) k_to_inner(int N, const double *__restrict__ r, float *__restrict__ r32,
                                                  float *__restrict__ d32, double *part)
{
    __shared__ double red[BLK / 64];
    double v = 0.0;
    for (int i = blockIdx.x * BLK + threadIdx.x; i < N; i += gridDim.x * BLK) {
        const float ri = float(r[i]);
        r32[i] = ri;
        d32[i] = 0.0f;
        v += double(ri) * double(ri);
    }
    const double bs = block_sum_all(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// One block: state of an inner solve (tolerance relative to its rhs).
__global__ void __launch_bounds__(BLK) k_begin_inner(CGState *st, const double *part, int n, double rtol,
                                                     int max_iter, int k_first)
{
    __shared__ double red[BLK / 64];
    const double bb = sum_partials(part, n, red);
    if (threadIdx.x == 0) {
        const double bn = sqrt(bb);
        st->bnorm = bn;
        st->tol = rtol * bn;
        st->rr = bb;
        st->tt = 0.0;
        st->iter = 0;
        st->max_iter = max_iter;
        st->status = isfinite(bn) ? 0 : PM_EBREAKDOWN;
        st->done = (!isfinite(bn) || !(bn > 0.0) || max_iter <= 0) ? 1 : 0;
        st->k_first = k_first;
    }
}

// One block: the inner solve continues after an FP64 correction.  The
// residual was just replaced (its partials are in part); the tolerance is
// relative to it; iteration count, budget and search direction carry on.
__global__ void __launch_bounds__(BLK) k_resume_inner(CGState *st, const double *part, int n, double rtol,
                                                      int k_first)
{
    __shared__ double red[BLK / 64];
    const double bb = sum_partials(part, n, red);
    if (threadIdx.x == 0) {
        const double bn = sqrt(bb);
        st->tol = rtol * bn;
        st->rr = bb;
        st->status = isfinite(bn) ? 0 : PM_EBREAKDOWN;
        st->done = (!isfinite(bn) || !(bn > 0.0) || st->iter >= st->max_iter) ? 1 : 0;
        st->k_first = k_first;
    }
}

// x += d (the inner correction, in FP64).
__global__ void __launch_bounds__(BLK) k_correct(int N, double *__restrict__ x, const float *__restrict__ d32)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i < N) x[i] += double(d32[i]);
}

__global__ void __launch_bounds__(BLK) k_gather(int N, const int *__restrict__ new2old,
                                                const double *__restrict__ src, double *__restrict__ dst)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i < N) dst[i] = src[new2old[i]];
}

__global__ void __launch_bounds__(BLK) k_scatter(int N, const int *__restrict__ new2old,
                                                 const double *__restrict__ src, double *__restrict__ dst)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i < N) dst[new2old[i]] = src[i];
}

}  // namespace

// ======================================================================
// Handle

struct pm_handle {
    int dim = 0;
    int64_t N = 0, E = 0, n_free = 0;
    double alpha = 0.0, dt = 0.0;
    int32_t flags = 0;
    int variant = PM_VARIANT_TILED;
    int mixed_mode = PM_MIXED_KEEP_DIRECTION;
    int device = 0;
    // operator data (device)
    int *new2old = nullptr;
    int *n2e_off = nullptr, *n2e_ent = nullptr;
    int4 *conn = nullptr;
    double *coords = nullptr;   // SoA
    double *coef = nullptr;     // c_e, internal element order
    double *w = nullptr;        // beta c_e / (d! det_e)
    uint8_t *dir = nullptr;
    // tiles (device)
    int tile_nodes = 0, n_tiles = 0, max_local = 0, max_deg = 0, max_inst = 0, tile_class = -1;
    size_t lds_limit = 65536;
    int64_t n_inst = 0;
    int *t_halo_off = nullptr, *t_halo = nullptr, *t_inst_off = nullptr, *t_inst_elem = nullptr;
    int *t_node_off = nullptr;  // tile t owns internal nodes [t_node_off[t], t_node_off[t+1])
    uint2 *t_inst = nullptr;
    double *t_inst_w = nullptr;
    uint8_t *t_nflag = nullptr;
    // FP32 operator data and inner-CG vectors (PM_FP32_INNER)
    float *coords32 = nullptr, *w32 = nullptr, *t_inst_w32 = nullptr;
    float *r32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    float *p32[2] = {nullptr, nullptr};
    CGState *st_in = nullptr;
    CGState *hst_in = nullptr;
    // host bookkeeping of a mixed-precision solve run by a batch; it lives
    // with the handle so that a rebuilt batch continues the solve
    struct MixedSolve {
        int phase = 0;       // MX_IDLE, MX_RESIDUAL, MX_INNER, MX_FINISHED
        double rtol = 0.0, rel = 0.0;
        int max_iter = 0, iters = 0, n_outer = 0, status = 0, iter0 = 0;
    } mx;
    // CG vectors (device, internal order)
    double *b = nullptr, *x = nullptr, *r = nullptr, *q = nullptr, *t = nullptr;
    bool lumped = false;        // PM_MASS_LUMPED: diagonal (row-sum) mass matrix
    // periodic mesh (merged images): period per axis, 0 = open
    bool periodic = false;
    double period[3] = {0.0, 0.0, 0.0};
    // alpha = 0 and no Dirichlet node: the solve is posed in V_0
    bool singular = false;
    double *mw = nullptr;       // m_i = int phi_i
    double m_total = 0.0;       // |Omega| = sum_i m_i
    double *pbuf[2] = {nullptr, nullptr};
    double *part = nullptr;     // [apply partials | rr partials x2 | misc partials]
    int n_vblocks = 0, n_ablocks = 0, n_ablocks32 = 0, n_cu = 256;
    CGState *st = nullptr;
    double *hist = nullptr;
    int32_t hist_cap = 0;
    CGState *hst = nullptr;     // pinned host mirror
    double *hist_host = nullptr;   // pinned host copy of the history (one-launch solves)
    int32_t hist_host_cap = 0;
    bool in_noalloc = false;       // inside pressure_solve_noalloc: allocate nothing
    size_t dev_bytes = 0;
    std::vector<int32_t> elem_new2old;   // host copy, for coefficient updates
    // projection stage: dual cells (built at the first use) and buffers
    struct Proj {
        bool built = false;
        pm::Faces F;                // counts (the lists are dropped after the upload)
        std::vector<int32_t> fv_caller, fe_caller;   // per face: caller node ids, caller elements
        int *efc = nullptr;         // 4 per internal element: face opposite internal-local vertex a
        int2 *fel = nullptr;        // per face: internal elements
        int *enew2old = nullptr;    // caller element of each internal element
        uint8_t *ebnd = nullptr;    // boundary-face bits per internal element
        int2 *fsl = nullptr;        // per face: element slots 4k + a (-1)
        int4 *trec = nullptr;       // transport records, 2 per (face, side); built on the first transport
        double *grad = nullptr;     // LADER: element gradients of rho and W_u; allocated on the first LADER step
        double *slots = nullptr;    // LADER: slot records (5 sums + volume share) per (element, face); idem
        int *oslot = nullptr;       // LADER: the other slot of each element slot's cell; idem
        double *contrib = nullptr;  // 4 per element: right-hand-side contributions
        double *e = nullptr;        // erho | ewe | erk | evol | ewu (x3) | egrad (x3), per element
        double *pn = nullptr, *gd = nullptr, *b = nullptr, *dp = nullptr, *dpi = nullptr;
    } pj;
    // timing (sampled: every TIMING_STRIDE-th apply launch of a solve)
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int64_t t_launches = 0;
    double t_ms = 0.0;

    double *part_pq() const { return part; }
    double *part_rr(int parity) const { return part + AGRID_MAX + parity * VGRID_MAX; }
    double *part_misc() const { return part + AGRID_MAX + 2 * VGRID_MAX; }
};

namespace {

constexpr int TIMING_STRIDE = 32;

// A failed HIP call returns PM_EHIP; with the environment variable
// PM_DEBUG set, the call, its source line and HIP's message go to stderr.
int hip_failed(hipError_t e, const char *what, int line)
{
    static const bool debug = std::getenv("PM_DEBUG") != nullptr;
    if (debug) std::fprintf(stderr, "libpressure: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
    return PM_EHIP;
}

#define HIPCK(x)                                                        \
    do {                                                                \
        const hipError_t hipck_e = (x);                                 \
        if (hipck_e != hipSuccess) return hip_failed(hipck_e, #x, __LINE__); \
    } while (0)

#define TRY(x)                      \
    do {                            \
        int _s = (x);               \
        if (_s != PM_OK) return _s; \
    } while (0)

template <class T>
int dalloc(pm_handle *h, T **p, size_t count)
{
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? PM_ENOMEM : PM_EHIP;
    }
    h->dev_bytes += bytes;
    return PM_OK;
}

// Setup work (uploads, clears, setup kernels) runs on a private non-blocking
// stream of the calling thread while a SetupStream is alive, so that a setup
// on one host thread neither waits for nor disturbs the streams of another
// (a graph capture there, for one: the legacy default stream would tie into
// it); the stream is drained before the setup call returns.
thread_local hipStream_t g_setup = nullptr;

struct SetupStream {
    bool owner = false;
    int status = PM_OK;
    SetupStream()
    {
        if (g_setup) return;   // nested: the outer call's stream
        if (hipStreamCreateWithFlags(&g_setup, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            g_setup = nullptr;
            status = PM_EHIP;
            return;
        }
        owner = true;
    }
    int finish()
    {
        if (owner && g_setup && hipStreamSynchronize(g_setup) != hipSuccess) return PM_EHIP;
        return PM_OK;
    }
    ~SetupStream()
    {
        if (!owner) return;
        (void)hipStreamSynchronize(g_setup);
        (void)hipStreamDestroy(g_setup);
        g_setup = nullptr;
    }
};

// host -> device (or device -> host) copy that is complete on return
int hcopy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    if (bytes == 0) return PM_OK;
    if (!g_setup) {
        HIPCK(hipMemcpy(dst, src, bytes, kind));
        return PM_OK;
    }
    HIPCK(hipMemcpyAsync(dst, src, bytes, kind, g_setup));
    HIPCK(hipStreamSynchronize(g_setup));
    return PM_OK;
}

// zero device memory, in setup-stream order
int hzero(void *p, size_t bytes)
{
    if (g_setup) HIPCK(hipMemsetAsync(p, 0, bytes, g_setup));
    else HIPCK(hipMemset(p, 0, bytes));
    return PM_OK;
}

template <class T>
int dupload(pm_handle *h, T **p, const std::vector<T> &v)
{
    TRY(dalloc(h, p, v.size()));
    if (!v.empty()) TRY(hcopy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return PM_OK;
}

inline unsigned grid_of(int64_t n) { return unsigned((n + BLK - 1) / BLK); }

// Mass coefficients of elem_contrib: consistent, alpha / (d! (d+1) (d+2))
// for both; lumped, alpha / (d! (d+1)) for x_a and 0 for S.
void mass_coefs(const pm_handle *h, double *mdiag, double *mfull)
{
    const double dfact = (h->dim == 2) ? 2.0 : 6.0;
    if (h->lumped) {
        *mdiag = h->alpha / (dfact * (h->dim + 1));
        *mfull = 0.0;
    } else {
        *mdiag = *mfull = h->alpha / (dfact * (h->dim + 1) * (h->dim + 2));
    }
}

template <class R>
MeshT<R> make_mesh(const pm_handle *h);

template <>
MeshT<double> make_mesh<double>(const pm_handle *h)
{
    MeshT<double> g;
    g.N = int(h->N);
    g.E = int(h->E);
    g.conn = h->conn;
    g.X = h->coords;
    g.Y = h->coords + h->N;
    g.Z = (h->dim == 3) ? h->coords + 2 * h->N : h->coords;
    g.w = h->w;
    g.dir = h->dir;
    mass_coefs(h, &g.mdiag, &g.mfull);
    for (int ax = 0; ax < 3; ++ax) {
        g.per[ax] = h->period[ax];
        g.iper[ax] = h->period[ax] > 0.0 ? 1.0 / h->period[ax] : 0.0;
    }
    return g;
}

template <>
MeshT<float> make_mesh<float>(const pm_handle *h)
{
    MeshT<float> g;
    g.N = int(h->N);
    g.E = int(h->E);
    g.conn = h->conn;
    g.X = h->coords32;
    g.Y = h->coords32 + h->N;
    g.Z = (h->dim == 3) ? h->coords32 + 2 * h->N : h->coords32;
    g.w = h->w32;
    g.dir = h->dir;
    double md, mf;
    mass_coefs(h, &md, &mf);
    g.mdiag = float(md);
    g.mfull = float(mf);
    for (int ax = 0; ax < 3; ++ax) {
        g.per[ax] = float(h->period[ax]);
        g.iper[ax] = h->period[ax] > 0.0 ? float(1.0 / h->period[ax]) : 0.0f;
    }
    return g;
}

template <class R>
TileArgsT<R> make_tiles(const pm_handle *h)
{
    TileArgsT<R> ta;
    ta.n_tiles = h->n_tiles;
    ta.max_deg = h->max_deg;
    ta.node_off = h->t_node_off;
    ta.halo_off = h->t_halo_off;
    ta.halo = h->t_halo;
    ta.inst_off = h->t_inst_off;
    ta.inst = h->t_inst;
    if constexpr (sizeof(R) == 8)
        ta.inst_w = h->t_inst_w;
    else
        ta.inst_w = h->t_inst_w32;
    ta.nflag = h->t_nflag;
    return ta;
}

bool valid_coef(const double *c, int64_t E)
{
    for (int64_t e = 0; e < E; ++e)
        if (!(c[e] > 0.0) || !std::isfinite(c[e])) return false;
    return true;
}

template <class R>
int compute_factors_t(pm_handle *h, R *w, R *inst_w, hipStream_t s)
{
    MeshT<R> g = make_mesh<R>(h);
    const double beta = h->dt * h->dt;
    const dim3 grid(grid_of(h->E));
    if (h->dim == 2 && h->periodic)
        hipLaunchKernelGGL((k_factors<2, R, true>), grid, dim3(BLK), 0, s, g, h->coef, beta, w);
    else if (h->dim == 2)
        hipLaunchKernelGGL((k_factors<2, R, false>), grid, dim3(BLK), 0, s, g, h->coef, beta, w);
    else if (h->periodic)
        hipLaunchKernelGGL((k_factors<3, R, true>), grid, dim3(BLK), 0, s, g, h->coef, beta, w);
    else
        hipLaunchKernelGGL((k_factors<3, R, false>), grid, dim3(BLK), 0, s, g, h->coef, beta, w);
    HIPCK(hipGetLastError());
    if (h->n_inst > 0) {
        hipLaunchKernelGGL(k_inst_factors<R>, dim3(grid_of(h->n_inst)), dim3(BLK), 0, s, int(h->n_inst),
                           h->t_inst_elem, w, inst_w);
        HIPCK(hipGetLastError());
    }
    return PM_OK;
}

// Per-instance copies of the FP64 element factors (after a kernel wrote w
// itself), and the FP32 factors if the handle has them, in stream order.
int refresh_factors_after_w(pm_handle *h, hipStream_t s)
{
    if (h->n_inst > 0) {
        hipLaunchKernelGGL(k_inst_factors<double>, dim3(grid_of(h->n_inst)), dim3(BLK), 0, s, int(h->n_inst),
                           h->t_inst_elem, h->w, h->t_inst_w);
        HIPCK(hipGetLastError());
    }
    if (h->w32) TRY(compute_factors_t<float>(h, h->w32, h->t_inst_w32, s));
    return PM_OK;
}

// Element factors from the current c_e, alpha and dt, in stream order.
int compute_factors_on(pm_handle *h, hipStream_t s)
{
    TRY(compute_factors_t<double>(h, h->w, h->t_inst_w, s));
    if (h->w32) TRY(compute_factors_t<float>(h, h->w32, h->t_inst_w32, s));
    return PM_OK;
}

int compute_factors(pm_handle *h)
{
    TRY(compute_factors_on(h, g_setup));
    if (g_setup) HIPCK(hipStreamSynchronize(g_setup));
    else HIPCK(hipDeviceSynchronize());
    return PM_OK;
}

template <class R>
size_t tiled_lds_bytes(int dim, int c, int max_deg)
{
    const TileClass tc = TILE_CLASSES[c];
    switch (tc.t) {
    case 128: return tile_lds_bytes<R, 128>(dim, tc.lm, max_deg);
    case 256: return tile_lds_bytes<R, 256>(dim, tc.lm, max_deg);
    default: return tile_lds_bytes<R, 512>(dim, tc.lm, max_deg);
    }
}

template <class R>
size_t tiled_lds_bytes(const pm_handle *h)
{
    return tiled_lds_bytes<R>(h->dim, h->tile_class, h->max_deg);
}

// Events of the next apply launch to time (start and stop are recorded by
// the command processor at the kernel's begin and end), or null.
thread_local hipEvent_t g_time_start = nullptr, g_time_stop = nullptr;

template <class R, class K>
int launch_tiled_k(pm_handle *h, K kern, int nth, const MeshT<R> &g, const TileArgsT<R> &ta, const R *x, R *y,
                   const IterT<R> &it, hipStream_t s)
{
    const size_t lds = tiled_lds_bytes<R>(h);
    if (lds > 65536) HIPCK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    const int grid = (sizeof(R) == 8) ? h->n_ablocks : h->n_ablocks32;
    if (g_time_start) {
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(nth), uint32_t(lds), s, g_time_start, g_time_stop, 0u, g, ta, x,
                              y, it);
        g_time_start = g_time_stop = nullptr;
    } else {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nth), lds, s, g, ta, x, y, it);
    }
    HIPCK(hipGetLastError());
    return PM_OK;
}

template <int DIM, bool CG, class R, int C>
int launch_tiled_c(pm_handle *h, const R *x, R *y, const IterT<R> &it, hipStream_t s)
{
    constexpr TileClass tc = TILE_CLASSES[C];
    MeshT<R> g = make_mesh<R>(h);
    TileArgsT<R> ta = make_tiles<R>(h);
    if (h->periodic)
        return launch_tiled_k<R>(h, k_apply_tiled<DIM, CG, R, tc.t, tc.ipt, tc.lm, tc.nth, true>, tc.nth, g, ta, x,
                                 y, it, s);
    return launch_tiled_k<R>(h, k_apply_tiled<DIM, CG, R, tc.t, tc.ipt, tc.lm, tc.nth, false>, tc.nth, g, ta, x, y,
                             it, s);
}

// f.template operator()<C>() for the handle's class C
template <class F>
int with_class(int c, F &&f)
{
    switch (c) {
    case 0: return f.template operator()<0>();
    case 1: return f.template operator()<1>();
    case 2: return f.template operator()<2>();
    case 3: return f.template operator()<3>();
    case 4: return f.template operator()<4>();
    case 5: return f.template operator()<5>();
    case 6: return f.template operator()<6>();
    case 7: return f.template operator()<7>();
    case 8: return f.template operator()<8>();
    case 9: return f.template operator()<9>();
    case 10: return f.template operator()<10>();
    case 11: return f.template operator()<11>();
    case 12: return f.template operator()<12>();
    default: return PM_EINVAL;
    }
}
static_assert(N_TILE_CLASSES == 13, "with_class covers every class");

template <int DIM, bool CG, class R>
int launch_tiled_t(pm_handle *h, const R *x, R *y, const IterT<R> &it, hipStream_t s)
{
    return with_class(h->tile_class, [&]<int C>() { return launch_tiled_c<DIM, CG, R, C>(h, x, y, it, s); });
}

// Resident blocks per CU of the CG apply kernel of the handle's size class.
template <int DIM, class R>
int occupancy_t(pm_handle *h, int *per_cu)
{
    return with_class(h->tile_class, [&]<int C>() {
        constexpr TileClass tc = TILE_CLASSES[C];
        const void *kern = h->periodic ? (const void *)k_apply_tiled<DIM, true, R, tc.t, tc.ipt, tc.lm, tc.nth, true>
                                       : (const void *)k_apply_tiled<DIM, true, R, tc.t, tc.ipt, tc.lm, tc.nth, false>;
        const size_t lds = tiled_lds_bytes<R>(h);
        if (lds > 65536) HIPCK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, tc.nth, lds));
        return PM_OK;
    });
}

// Grid of the tiled apply: every block resident at once (one per resident
// slot over all CUs), a multiple of the XCD count, at most one per tile.
template <class R>
int apply_grid(pm_handle *h, int *grid)
{
    int per_cu = 0;
    const int st = (h->dim == 2) ? occupancy_t<2, R>(h, &per_cu) : occupancy_t<3, R>(h, &per_cu);
    if (st != PM_OK) return st;
    int g = std::max(1, per_cu) * h->n_cu;
    g = std::min(g, AGRID_MAX);
    if (g >= N_XCD) g -= g % N_XCD;
    *grid = std::max(1, std::min(g, h->n_tiles));
    return PM_OK;
}

template <int DIM, bool CG>
int launch_node_t(pm_handle *h, const double *x, double *y, const Iter &it, hipStream_t s)
{
    Mesh g = make_mesh<double>(h);
    if (h->periodic)
        hipLaunchKernelGGL((k_apply_node<DIM, CG, true>), dim3(h->n_ablocks), dim3(BLK), 0, s, g, h->n2e_off,
                           h->n2e_ent, h->t_node_off, h->n_tiles, x, y, it);
    else
        hipLaunchKernelGGL((k_apply_node<DIM, CG, false>), dim3(h->n_ablocks), dim3(BLK), 0, s, g, h->n2e_off,
                           h->n2e_ent, h->t_node_off, h->n_tiles, x, y, it);
    HIPCK(hipGetLastError());
    return PM_OK;
}

// y = A x on internal vectors (cg = false) or one CG iteration's apply.
int launch_apply(pm_handle *h, const double *x, double *y, const Iter *it, hipStream_t s)
{
    Iter dummy{};
    const Iter &a = it ? *it : dummy;
    const bool cg = it != nullptr;
    if (h->variant == PM_VARIANT_NODE) {
        if (h->dim == 2) return cg ? launch_node_t<2, true>(h, x, y, a, s) : launch_node_t<2, false>(h, x, y, a, s);
        return cg ? launch_node_t<3, true>(h, x, y, a, s) : launch_node_t<3, false>(h, x, y, a, s);
    }
    if (h->dim == 2)
        return cg ? launch_tiled_t<2, true, double>(h, x, y, a, s) : launch_tiled_t<2, false, double>(h, x, y, a, s);
    return cg ? launch_tiled_t<3, true, double>(h, x, y, a, s) : launch_tiled_t<3, false, double>(h, x, y, a, s);
}

// One FP32 inner-CG iteration's apply (tiled kernel only).
int launch_apply32(pm_handle *h, const IterT<float> &it, hipStream_t s)
{
    if (h->dim == 2) return launch_tiled_t<2, true, float>(h, it.p_new, it.q, it, s);
    return launch_tiled_t<3, true, float>(h, it.p_new, it.q, it, s);
}

int ensure_hist(pm_handle *h, int32_t max_iter)
{
    if (max_iter + 1 <= h->hist_cap) return PM_OK;
    if (h->hist) {
        HIPCK(hipFree(h->hist));
        h->dev_bytes -= size_t(h->hist_cap) * sizeof(double);
        h->hist = nullptr;
    }
    int32_t cap = std::max<int32_t>(max_iter + 1, 1024);
    TRY(dalloc(h, &h->hist, size_t(cap)));
    h->hist_cap = cap;
    return PM_OK;
}

// The pinned host history of the one-launch solve, or nullptr when the
// call may not allocate and the buffer is too small.
static int ensure_hist_host(pm_handle *h, int32_t max_iter, double **out)
{
    *out = nullptr;
    if (max_iter + 1 > h->hist_host_cap) {
        if (h->in_noalloc) return PM_OK;
        if (h->hist_host) HIPCK(hipHostFree(h->hist_host));
        h->hist_host = nullptr;
        h->hist_host_cap = 0;
        const int32_t cap = std::max<int32_t>(max_iter + 1, 1024);
        HIPCK(hipHostMalloc((void **)&h->hist_host, sizeof(double) * size_t(cap), hipHostMallocDefault));
        h->hist_host_cap = cap;
    }
    *out = h->hist_host;
    return PM_OK;
}

int event_pair(pm_handle *h, size_t k, hipEvent_t *a, hipEvent_t *b)
{
    while (h->ev.size() < 2 * (k + 1)) {
        hipEvent_t e;
        HIPCK(hipEventCreate(&e));
        h->ev.push_back(e);
    }
    *a = h->ev[2 * k];
    *b = h->ev[2 * k + 1];
    return PM_OK;
}

// Tiles of the tiled apply.  Returns pm::TILES_TOO_WIDE when the mesh does
// not fit the tiled kernel at this tile size (a node with more elements, or
// a tile with more own and halo nodes, than a record names; no size class
// or not enough LDS for the largest tile).
// Smallest size class of this tile size that covers the tiles' instances
// and node tables, or -1.
int pick_class(int tile_nodes, int max_inst, int max_local)
{
    for (int c = 0; c < N_TILE_CLASSES; ++c)
        if (TILE_CLASSES[c].t == tile_nodes && TILE_CLASSES[c].ipt * TILE_CLASSES[c].nth >= max_inst &&
            TILE_CLASSES[c].lm >= max_local)
            return c;
    return -1;
}

void adopt_tiles(pm_handle *h, const pm::Tiles &T, int tile_nodes)
{
    h->tile_nodes = tile_nodes;
    h->n_tiles = int(T.n_tiles);
    h->max_local = tile_nodes + T.max_halo;
    h->max_deg = T.max_deg;
    h->max_inst = T.max_inst;
    h->n_inst = int64_t(T.inst_elem.size());
    h->tile_class = pick_class(tile_nodes, T.max_inst, h->max_local);
}

int build_tiles_on_device(pm_handle *h, const pm::Layout &L, int tile_nodes)
{
    pm::Tiles T;
    TRY(pm::build_tiles(L, tile_nodes, &T));
    adopt_tiles(h, T, tile_nodes);
    if (h->tile_class < 0 || tiled_lds_bytes<double>(h) > h->lds_limit) {
        h->tile_class = -1;
        return pm::TILES_TOO_WIDE;
    }
    std::vector<uint8_t> nflag(L.n_nodes);
    for (int64_t i = 0; i < L.n_nodes; ++i)
        nflag[i] = uint8_t((L.n2e_off[i + 1] - L.n2e_off[i]) | (L.dirichlet[i] ? 0x80 : 0));
    TRY(dupload(h, &h->t_node_off, T.node_off));
    TRY(dupload(h, &h->t_halo_off, T.halo_off));
    {
        // halo ids carry the Dirichlet flag in bit 31
        std::vector<int32_t> hal(T.halo);
        for (auto &v : hal)
            if (L.dirichlet[v]) v = int32_t(uint32_t(v) | DIR_BIT);
        TRY(dupload(h, &h->t_halo, hal));
    }
    TRY(dupload(h, &h->t_inst_off, T.inst_off));
    TRY(dupload(h, &h->t_inst_elem, T.inst_elem));
    TRY(dupload(h, &h->t_nflag, nflag));
    TRY(dalloc(h, &h->t_inst, size_t(h->n_inst)));
    if (h->n_inst > 0)
        TRY(hcopy(h->t_inst, T.inst.data(), sizeof(uint16_t) * T.inst.size(), hipMemcpyHostToDevice));
    TRY(dalloc(h, &h->t_inst_w, size_t(h->n_inst)));
    TRY(apply_grid<double>(h, &h->n_ablocks));
    return PM_OK;
}

// Meshes the tiled kernel does not take (see build_tiles_on_device) run on
// the node kernel alone, over 128-node runs in the same block order.
int setup_node_only(pm_handle *h)
{
    h->variant = PM_VARIANT_NODE;
    h->tile_class = -1;
    h->tile_nodes = 128;
    h->n_tiles = int((h->N + 127) / 128);
    h->n_inst = 0;
    h->max_inst = 0;
    std::vector<int32_t> off(h->n_tiles + 1);
    for (int64_t t = 0; t <= h->n_tiles; ++t) off[t] = int32_t(std::min<int64_t>(h->N, 128 * t));
    TRY(dupload(h, &h->t_node_off, off));
    int g = std::min(AGRID_MAX, 8 * h->n_cu);
    if (g >= N_XCD) g -= g % N_XCD;
    h->n_ablocks = std::max(1, std::min(g, h->n_tiles));
    return PM_OK;
}

}  // namespace

// ======================================================================
// Static scratch of pressure_solve_noalloc: the CG vectors, block partials,
// solver state and residual history of one FP64 solve of up to
// PM_NOALLOC_MAX_NODES nodes and PM_NOALLOC_MAX_ITER iterations, in a
// file-scope device array, so that the call allocates nothing.  Every GPU
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is not a device address on the host).
// Layout (doubles): b | x | r | q | p_0 | p_1 (one PM_NOALLOC_MAX_NODES
// stride each), block partials, history, solver state.

namespace {
constexpr size_t NA_VEC = size_t(PM_NOALLOC_MAX_NODES);
constexpr size_t NA_PART = size_t(AGRID_MAX + 3 * VGRID_MAX);
constexpr size_t NA_HIST = size_t(PM_NOALLOC_MAX_ITER) + 1;
constexpr size_t NA_STATE = (sizeof(CGState) + 7) / 8;
constexpr size_t NA_DOUBLES = 6 * NA_VEC + NA_PART + NA_HIST + NA_STATE;
}  // namespace

static __device__ __align__(256) double scratch[NA_DOUBLES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NA_MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up once per device
// (the caller has made `device` current).
int noalloc_scratch_init(int device)
{
    if (device < 0 || device >= NA_MAX_DEVICES) return PM_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return PM_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return PM_EHIP;
    }
    g_scratch_ptr[device] = static_cast<double *>(ptr);
    return PM_OK;
}

double *noalloc_scratch(int device)
{
    if (device < 0 || device >= NA_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

__global__ void k_fill2(int64_t n, double *a, double *b, double v)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        a[i] = v;
        b[i] = v;
    }
}

// The handle's solve buffers, swapped for the scratch for one call and put
// back on every return path.
struct ScratchSwap {
    pm_handle *h;
    double *b, *x, *r, *q, *p0, *p1, *part, *hist;
    CGState *st;
    int32_t hist_cap;
    bool timing;
    ScratchSwap(pm_handle *hh, double *base) : h(hh)
    {
        b = h->b, x = h->x, r = h->r, q = h->q, p0 = h->pbuf[0], p1 = h->pbuf[1];
        part = h->part, hist = h->hist, st = h->st, hist_cap = h->hist_cap, timing = h->timing;
        h->b = base;
        h->x = base + NA_VEC;
        h->r = base + 2 * NA_VEC;
        h->q = base + 3 * NA_VEC;
        h->pbuf[0] = base + 4 * NA_VEC;
        h->pbuf[1] = base + 5 * NA_VEC;
        h->part = base + 6 * NA_VEC;
        h->hist = h->part + NA_PART;
        h->hist_cap = int32_t(NA_HIST);
        h->st = reinterpret_cast<CGState *>(h->hist + NA_HIST);
        h->timing = false;   // timing events would be created on demand
        h->in_noalloc = true;
    }
    ~ScratchSwap()
    {
        h->b = b, h->x = x, h->r = r, h->q = q, h->pbuf[0] = p0, h->pbuf[1] = p1;
        h->part = part, h->hist = hist, h->st = st, h->hist_cap = hist_cap, h->timing = timing;
        h->in_noalloc = false;
    }
};
}  // namespace

// ======================================================================
// C ABI

extern "C" {

const char *pressure_strerror(int status)
{
    switch (status) {
    case PM_OK: return "ok";
    case PM_NOT_CONVERGED: return "not converged within max_iter";
    case PM_EINVAL: return "invalid argument";
    case PM_EDEGENERATE: return "degenerate element (zero volume)";
    case PM_ENOMEM: return "out of memory";
    case PM_EBREAKDOWN: return "CG breakdown (p.Ap <= 0 or not finite)";
    case PM_EHIP: return "HIP runtime error";
    case PM_ETIMEOUT: return "a grid barrier of a persistent batched launch timed out";
    case PM_PENDING: return "the batch step is still running";
    case PM_ETOOLARGE:
        return "larger than the static scratch of pressure_solve_noalloc (n_nodes > PM_NOALLOC_MAX_NODES or "
               "max_iter > PM_NOALLOC_MAX_ITER)";
    default: return "unknown status";
    }
}

int pressure_layout(const pm_mesh *mesh, int32_t *node_new2old, int32_t *elem_new2old,
                    int32_t *elems_new, int32_t *n2e_off, int32_t *n2e_ent)
{
    try {
        pm::Layout L;
        int s = pm::build_layout(mesh, &L);
        if (s != PM_OK) return s;
        const int nv = L.dim + 1;
        if (node_new2old) std::memcpy(node_new2old, L.node_new2old.data(), sizeof(int32_t) * L.n_nodes);
        if (elem_new2old) std::memcpy(elem_new2old, L.elem_new2old.data(), sizeof(int32_t) * L.n_elems);
        if (elems_new)
            for (int64_t e = 0; e < L.n_elems; ++e)
                for (int a = 0; a < nv; ++a) elems_new[e * nv + a] = L.conn[e * 4 + a];
        if (n2e_off) std::memcpy(n2e_off, L.n2e_off.data(), sizeof(int32_t) * (L.n_nodes + 1));
        if (n2e_ent) std::memcpy(n2e_ent, L.n2e_ent.data(), sizeof(int32_t) * L.n2e_ent.size());
        return PM_OK;
    } catch (const std::bad_alloc &) {
        return PM_ENOMEM;
    } catch (...) {
        return PM_EINVAL;
    }
}

int pressure_footprint(const pm_mesh *mesh, int32_t flags, uint64_t *bytes)
{
    if (!mesh || !bytes || (mesh->dim != 2 && mesh->dim != 3) || mesh->n_nodes < 1 || mesh->n_elems < 1)
        return PM_EINVAL;
    (void)flags;
    const uint64_t N = uint64_t(mesh->n_nodes), E = uint64_t(mesh->n_elems), d = uint64_t(mesh->dim);
    // element instances over all tiles: at most 2 x elements on the meshes of
    // interest (measured 1.3-1.6 x on Morton tiles of 256-1024 nodes)
    const uint64_t I = 2 * E;
    uint64_t b = 0;
    b += 4 * N;                             // new2old
    b += 4 * (N + 1) + 4 * (d + 1) * E;     // node-to-element lists
    b += 16 * E;                            // connectivity
    b += 8 * d * N;                         // coordinates
    b += 16 * E;                            // c_e and w_e
    b += N;                                 // Dirichlet flags
    b += I * (8 + 8 + 4) + 8 * N + 8 * N;   // tiles: records, factors, element ids; halo lists, flags
    b += 4 * (N / 64 + 2);                  // tile node ranges
    b += 7 * 8 * N;                         // b, x, r, q, t, p (x2)
    b += 8 * (AGRID_MAX + 3 * VGRID_MAX) + 1024 * 8 + 256;
    if (flags & PM_FP32_INNER)   // FP32 coordinates, factors and inner-CG vectors
        b += 4 * d * N + 4 * E + 4 * I + 5 * 4 * N + 256;
    *bytes = b;
    return PM_OK;
}

void pressure_destroy(pm_handle *h)
{
    if (!h) return;
    void *ptrs[] = {h->new2old, h->n2e_off, h->n2e_ent, h->conn, h->coords, h->coef, h->w, h->dir,
                    h->t_halo_off, h->t_halo, h->t_inst_off, h->t_inst_elem, h->t_inst, h->t_inst_w, h->t_node_off,
                    h->t_nflag, h->b, h->x, h->r, h->q, h->t, h->pbuf[0],
                    h->pbuf[1], h->part, h->st, h->hist, h->coords32, h->w32, h->t_inst_w32, h->r32, h->q32,
                    h->d32, h->p32[0], h->p32[1], h->st_in, h->mw, h->pj.efc, h->pj.fel, h->pj.enew2old,
                    h->pj.e, h->pj.pn, h->pj.gd, h->pj.b, h->pj.dp, h->pj.dpi, h->pj.ebnd, h->pj.contrib, h->pj.fsl, h->pj.trec, h->pj.grad,
                    h->pj.slots, h->pj.oslot};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (h->hst) (void)hipHostFree(h->hst);
    if (h->hist_host) (void)hipHostFree(h->hist_host);
    if (h->hst_in) (void)hipHostFree(h->hst_in);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    delete h;
}

// No Dirichlet node and alpha = 0: the solve is posed in V_0, which needs the
// lumped mass weights m_i = int phi_i and |Omega| (computed once).
static int update_v0(pm_handle *h)
{
    h->singular = (h->n_free == h->N && h->alpha == 0.0);
    if (!h->singular || h->mw) return PM_OK;
    const int64_t N = h->N;
    TRY(dalloc(h, &h->mw, N));
    Mesh g = make_mesh<double>(h);
    const dim3 grid(grid_of(N));
    if (h->dim == 2 && h->periodic)
        hipLaunchKernelGGL((k_lumped_mass<2, true>), grid, dim3(BLK), 0, g_setup, g, h->n2e_off, h->n2e_ent, h->mw);
    else if (h->dim == 2)
        hipLaunchKernelGGL((k_lumped_mass<2, false>), grid, dim3(BLK), 0, g_setup, g, h->n2e_off, h->n2e_ent, h->mw);
    else if (h->periodic)
        hipLaunchKernelGGL((k_lumped_mass<3, true>), grid, dim3(BLK), 0, g_setup, g, h->n2e_off, h->n2e_ent, h->mw);
    else
        hipLaunchKernelGGL((k_lumped_mass<3, false>), grid, dim3(BLK), 0, g_setup, g, h->n2e_off, h->n2e_ent, h->mw);
    HIPCK(hipGetLastError());
    std::vector<double> mw(N);
    TRY(hcopy(mw.data(), h->mw, 8 * N, hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (double v : mw) tot += v;
    h->m_total = tot;
    return PM_OK;
}

static int tile_nodes_for(int32_t flags)
{
    switch (flags & PM_TILE_MASK) {
    case PM_TILE_256: return 256;
    case PM_TILE_512: return 512;
    case PM_TILE_128: return 128;
    case 0: return 128;
    default: return -1;
    }
}

static int setup_impl(const pm_mesh *mesh, const double *elem_coef, double mass_coef, double dt,
                      int32_t flags, pm_handle *h)
{
    if (!elem_coef || !(mass_coef >= 0.0) || !std::isfinite(mass_coef) || !(dt > 0.0) || !std::isfinite(dt))
        return PM_EINVAL;
    if (flags & ~(PM_FP64 | PM_FP32_INNER | PM_TILE_MASK | PM_MASS_LUMPED)) return PM_EINVAL;
    if (!mesh || !valid_coef(elem_coef, mesh->n_elems)) return PM_EINVAL;
    pm::Layout L;
    TRY(pm::build_layout(mesh, &L));
    HIPCK(hipGetDevice(&h->device));
    TRY(noalloc_scratch_init(h->device));
    {
        int v = 0;
        HIPCK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
        h->lds_limit = size_t(v) - 1024;   // static LDS of the kernels
        HIPCK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, h->device));
        h->n_cu = std::max(1, v);
    }
    h->dim = L.dim;
    h->N = L.n_nodes;
    h->E = L.n_elems;
    h->n_free = L.n_free;
    h->periodic = L.periodic;
    for (int ax = 0; ax < 3; ++ax) h->period[ax] = L.period[ax];
    h->alpha = mass_coef;
    h->dt = dt;
    h->flags = flags;
    h->lumped = (flags & PM_MASS_LUMPED) != 0;
    const int64_t N = h->N, E = h->E;
    // vector kernels: about 4 nodes per lane (fewer blocks also means fewer
    // partials for the next kernel's prologue to sum)
    h->n_vblocks = int(std::max<int64_t>(1, std::min<int64_t>((N + 4 * BLK - 1) / (4 * BLK), VGRID_MAX)));

    // connectivity with the Dirichlet flag of each vertex in bit 31
    std::vector<int32_t> conn(L.conn);
    const int nv = L.dim + 1;
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nv; ++a) {
            int32_t v = conn[e * 4 + a];
            if (L.dirichlet[v]) conn[e * 4 + a] = int32_t(uint32_t(v) | DIR_BIT);
        }
    std::vector<double> cnew(E);
    for (int64_t e = 0; e < E; ++e) cnew[e] = elem_coef[L.elem_new2old[e]];
    h->elem_new2old = L.elem_new2old;

    TRY(dupload(h, &h->new2old, L.node_new2old));
    TRY(dupload(h, &h->n2e_off, L.n2e_off));
    TRY(dupload(h, &h->n2e_ent, L.n2e_ent));
    TRY(dalloc(h, &h->conn, E));
    TRY(hcopy(h->conn, conn.data(), 16 * E, hipMemcpyHostToDevice));
    TRY(dupload(h, &h->coords, L.coords));
    TRY(dupload(h, &h->coef, cnew));
    TRY(dalloc(h, &h->w, E));
    TRY(dupload(h, &h->dir, L.dirichlet));
    const int tn = tile_nodes_for(flags);
    if (tn < 0) return PM_EINVAL;
    {
        int st = build_tiles_on_device(h, L, tn);
        if (st == pm::TILES_TOO_WIDE) {
            // an explicit tile size is an error; the default runs the node kernel
            if ((flags & PM_TILE_MASK) != 0 || (flags & PM_FP32_INNER)) return PM_EINVAL;
            st = setup_node_only(h);
        }
        TRY(st);
    }
    for (double **v : {&h->b, &h->x, &h->r, &h->q, &h->t, &h->pbuf[0], &h->pbuf[1]}) TRY(dalloc(h, v, N));
    if (flags & PM_FP32_INNER) {
        std::vector<float> c32(L.coords.size());
        for (size_t i = 0; i < c32.size(); ++i) c32[i] = float(L.coords[i]);
        TRY(dupload(h, &h->coords32, c32));
        TRY(dalloc(h, &h->w32, E));
        TRY(dalloc(h, &h->t_inst_w32, size_t(std::max<int64_t>(h->n_inst, 1))));
        for (float **v : {&h->r32, &h->q32, &h->d32, &h->p32[0], &h->p32[1]}) TRY(dalloc(h, v, N));
        TRY(hzero(h->p32[0], 4 * N));
        TRY(hzero(h->p32[1], 4 * N));
        TRY(dalloc(h, &h->st_in, 1));
        TRY(hzero(h->st_in, sizeof(CGState)));
        hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, g_setup, h->st_in);   // idle until a mixed solve starts
        HIPCK(hipHostMalloc((void **)&h->hst_in, sizeof(CGState), hipHostMallocDefault));
        if (tiled_lds_bytes<float>(h) > h->lds_limit) return PM_EINVAL;
        TRY(apply_grid<float>(h, &h->n_ablocks32));
    }
    TRY(dalloc(h, &h->part, AGRID_MAX + 3 * VGRID_MAX));
    TRY(dalloc(h, &h->st, 1));
    TRY(ensure_hist(h, 1023));
    HIPCK(hipHostMalloc((void **)&h->hst, sizeof(CGState), hipHostMallocDefault));
    TRY(hzero(h->st, sizeof(CGState)));
    hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, g_setup, h->st);   // idle until a solve starts
    HIPCK(hipGetLastError());
    TRY(hzero(h->part, sizeof(double) * (AGRID_MAX + 3 * VGRID_MAX)));
    TRY(hzero(h->pbuf[0], 8 * N));
    TRY(hzero(h->pbuf[1], 8 * N));
    TRY(compute_factors(h));
    return update_v0(h);
}

int pressure_setup(const pm_mesh *mesh, const double *elem_coef, double mass_coef, double dt,
                   int32_t flags, pm_handle **out)
{
    if (!out) return PM_EINVAL;
    *out = nullptr;
    pm_handle *h = nullptr;
    SetupStream ss;
    if (ss.status != PM_OK) return ss.status;
    try {
        h = new pm_handle();
        int s = setup_impl(mesh, elem_coef, mass_coef, dt, flags, h);
        if (s == PM_OK) s = ss.finish();
        if (s != PM_OK) {
            pressure_destroy(h);
            return s;
        }
    } catch (const std::bad_alloc &) {
        pressure_destroy(h);
        return PM_ENOMEM;
    } catch (...) {
        pressure_destroy(h);
        return PM_EINVAL;
    }
    *out = h;
    return PM_OK;
}

int pressure_update_coef(pm_handle *h, const double *elem_coef, double mass_coef, double dt)
{
    if (!h || !(mass_coef >= 0.0) || !std::isfinite(mass_coef) || !(dt > 0.0) || !std::isfinite(dt))
        return PM_EINVAL;
    SetupStream ss;
    if (ss.status != PM_OK) return ss.status;
    if (elem_coef) {
        if (!valid_coef(elem_coef, h->E)) return PM_EINVAL;
        std::vector<double> cnew(h->E);
        for (int64_t e = 0; e < h->E; ++e) cnew[e] = elem_coef[h->elem_new2old[e]];
        TRY(hcopy(h->coef, cnew.data(), 8 * h->E, hipMemcpyHostToDevice));
    }
    h->alpha = mass_coef;
    h->dt = dt;
    TRY(compute_factors(h));
    TRY(update_v0(h));
    return ss.finish();
}

int pressure_apply(pm_handle *h, const double *x_dev, double *y_dev, void *stream)
{
    if (!h || !x_dev || !y_dev || x_dev == y_dev) return PM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const unsigned grid = grid_of(h->N);
    const int N = int(h->N);
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(BLK), 0, s, N, h->new2old, x_dev, h->t);
    HIPCK(hipGetLastError());
    TRY(launch_apply(h, h->t, h->q, nullptr, s));
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(BLK), 0, s, N, h->new2old, h->q, y_dev);
    HIPCK(hipGetLastError());
    return PM_OK;
}

// Launch CG iterations k0 .. k0+count-1 (the first one with beta = 0 when
// first is set).
static int launch_iterations(pm_handle *h, int k0, int count, bool first, size_t *timed, hipStream_t s)
{
    const int N = int(h->N);
    for (int c = 0; c < count; ++c) {
        const int k = k0 + c;
        Iter it;
        it.k = k;
        it.first = (first && c == 0) ? 1 : 0;
        it.r = h->r;
        it.p_old = h->pbuf[(k - 1) & 1];
        it.p_new = h->pbuf[k & 1];
        it.q = h->q;
        it.st = h->st;
        it.hist = h->hist;
        it.part_pq = h->part_pq();
        it.rr_cur = h->part_rr((k - 1) & 1);
        it.rr_prev = h->part_rr(k & 1);
        it.n_vblocks = h->n_vblocks;
        const bool sample = h->timing && (k % TIMING_STRIDE) == 1 && h->variant != PM_VARIANT_NODE;
        if (sample) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            TRY(event_pair(h, *timed, &e0, &e1));
            g_time_start = e0;
            g_time_stop = e1;
            ++*timed;
        }
        TRY(launch_apply(h, it.p_new, h->q, &it, s));
        hipLaunchKernelGGL(k_update<double>, dim3(h->n_vblocks), dim3(BLK), 0, s, N, h->x, h->r, h->pbuf[k & 1], h->q,
                           h->st, h->part_pq(), h->n_ablocks, h->part_rr((k - 1) & 1), h->n_vblocks,
                           h->part_rr(k & 1));
    }
    HIPCK(hipGetLastError());
    return PM_OK;
}

// V_0 (singular handles only): b -= (sum b / |Omega|) m, with the partials of
// b.b for ||b|| where k_prepare left them; and, after the solve, the shift
// x -= (sum_i m_i x_i / |Omega|) that makes int x_h = 0.
static int project_rhs(pm_handle *h, hipStream_t s)
{
    if (!h->singular) return PM_OK;
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;
    hipLaunchKernelGGL(k_wsum, dim3(vg), dim3(BLK), 0, s, N, nullptr, h->b, h->part_rr(0));
    hipLaunchKernelGGL(k_sub_mean, dim3(vg), dim3(BLK), 0, s, N, h->b, h->mw, h->part_rr(0), int(vg), h->m_total,
                       h->part_misc());
    HIPCK(hipGetLastError());
    return PM_OK;
}

static int shift_mean(pm_handle *h, hipStream_t s)
{
    if (!h->singular) return PM_OK;
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;
    hipLaunchKernelGGL(k_wsum, dim3(vg), dim3(BLK), 0, s, N, h->mw, h->x, h->part_misc());
    hipLaunchKernelGGL(k_sub_mean, dim3(vg), dim3(BLK), 0, s, N, h->x, nullptr, h->part_misc(), int(vg), h->m_total,
                       nullptr);
    HIPCK(hipGetLastError());
    return PM_OK;
}

// Iterations to launch before the host looks at the state again: the
// number still needed at the residual's mean rate since the last look
// (plus 10 % and 2), within [4, 64]; doubling while no rate is known or the
// residual did not fall (the CG residual is not monotone).  Launches past
// convergence exit at once, so an overestimate costs little and an
// underestimate one more look.
static int next_chunk(const CGState &st, int chunk, double rr_seen, int it_seen)
{
    const int doubled = std::min(chunk * 2, 64);
    if (!(rr_seen > 0.0) || !(st.rr > 0.0) || !(st.rr < rr_seen) || st.iter <= it_seen) return doubled;
    const double rate = 0.5 * std::log(st.rr / rr_seen) / double(st.iter - it_seen);   // log of the factor per iteration
    const double need = std::log(st.tol / std::sqrt(st.rr)) / rate;
    if (!std::isfinite(need) || !(need > 0.0)) return doubled;
    return int(std::clamp(std::ceil(1.1 * need) + 2.0, 4.0, 64.0));
}

static int read_state(pm_handle *h, hipStream_t s)
{
    HIPCK(hipMemcpyAsync(h->hst, h->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    return PM_OK;
}

// The one-launch solve takes meshes whose data fit one block's LDS, on
// the tiled kernel's grids with one tile per apply block; sampled kernel
// timing needs the per-iteration launches.
static bool small_ok(const pm_handle *h)
{
    if (h->variant != PM_VARIANT_TILED || h->timing || h->tile_nodes != 128) return false;
    if (h->n_ablocks != h->n_tiles || h->n_tiles > 256 || h->n_vblocks > 4) return false;
    if (h->N > int64_t(SMALL_MPT) * BLK * h->n_vblocks || h->E > int64_t(small_ept(h->dim)) * SMALL_NTH) return false;
    return small_lds_bytes(h->dim, h->N, h->E, h->n_ablocks, h->n_tiles) <= size_t(h->lds_limit);
}

// One launch of the one-workgroup solve from iteration k0; with rhs set
// (k0 = 1) it also starts the solve from rhs and x0.
static int launch_small(pm_handle *h, int k0, const double *rhs, const double *x0, double rtol, int max_iter,
                        double *hist_host, CGState *st_host, hipStream_t s)
{
    const size_t lds = small_lds_bytes(h->dim, h->N, h->E, h->n_ablocks, h->n_tiles);
    Mesh g = make_mesh<double>(h);
    SmallArgs a;
    a.n2e_off = h->n2e_off;
    a.n2e_ent = h->n2e_ent;
    a.node_off = h->t_node_off;
    a.new2old = h->new2old;
    a.n_tiles = h->n_tiles;
    a.n_ablocks = h->n_ablocks;
    a.n_vblocks = h->n_vblocks;
    a.x = h->x;
    a.r = h->r;
    a.b = h->b;
    a.st = h->st;
    a.hist = h->hist;
    a.rr_parts = h->part_rr(0);
    a.k0 = k0;
    a.rhs = rhs;
    a.x0 = x0;
    a.rtol = rtol;
    a.max_iter = max_iter;
    a.hist_host = hist_host;
    a.st_host = st_host;
    auto go = [&]<int DIM, bool PER>() -> int {
        auto run = [&]<int EPT, bool GEO>() -> int {
            const void *kern = (const void *)k_solve_small<DIM, PER, EPT, GEO>;
            // the LDS limit is raised to the device's once per kernel and device
            static std::atomic<unsigned long long> raised{0};
            const unsigned long long bit = 1ull << (h->device & 63);
            if (lds > 65536 && !(raised.load() & bit)) {
                HIPCK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(h->lds_limit)));
                raised.fetch_or(bit);
            }
            hipLaunchKernelGGL((k_solve_small<DIM, PER, EPT, GEO>), dim3(1), dim3(SMALL_NTH), lds, s, g, a);
            HIPCK(hipGetLastError());
            return PM_OK;
        };
        if constexpr (DIM == 2)
            if (h->E <= int64_t(SMALL_GEO_EPT) * SMALL_NTH) return run.template operator()<SMALL_GEO_EPT, true>();
        return run.template operator()<small_ept(DIM), false>();
    };
    if (h->dim == 2) return h->periodic ? go.template operator()<2, true>() : go.template operator()<2, false>();
    return h->periodic ? go.template operator()<3, true>() : go.template operator()<3, false>();
}

int pressure_solve(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                   int32_t max_iter, double *p_dev, int32_t *iters, double *res_hist,
                   double *true_relres, void *stream)
{
    if (!h || !rhs_dev || !p_dev || !iters || !(rtol > 0.0) || !std::isfinite(rtol) || max_iter < 0)
        return PM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_hist(h, max_iter));
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;

    // A small mesh runs each pass of the solve (the start, the iterations
    // up to the stop, the true residual) in one launch; the first pass also
    // starts the solve unless the rhs must first be projected onto V_0.
    const bool small = small_ok(h);
    const bool small_start = small && !h->singular;
    double *hist_host = nullptr;   // set: the one-launch passes write the history and state to the host too
    if (small_start) TRY(ensure_hist_host(h, max_iter, &hist_host));
    if (!small_start) {
        hipLaunchKernelGGL(k_prepare, dim3(vg), dim3(BLK), 0, s, N, h->new2old, h->dir, rhs_dev, x0_dev, h->b, h->x,
                           h->part_misc());
        TRY(project_rhs(h, s));
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg), rtol, max_iter, h->hist,
                           1);
        HIPCK(hipGetLastError());
        TRY(launch_apply(h, h->x, h->q, nullptr, s));
        hipLaunchKernelGGL(k_start, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->x, h->r, h->st, h->part_rr(0));
        HIPCK(hipGetLastError());
    }

    int replaced = 0;
    int k = 1;            // next iteration to launch
    bool first = true;    // k is the first iteration after a (re)start
    size_t timed = 0;
    for (;;) {
        int chunk = 4;
        double rr_seen = -1.0;
        int it_seen = 0;
        if (small) {
            const bool with_start = small_start && k == 1 && replaced == 0;
            // the launch writes the history and the final state to pinned
            // host memory as well, so one synchronisation ends the pass
            TRY(launch_small(h, k, with_start ? rhs_dev : nullptr, x0_dev, rtol, max_iter, hist_host,
                             hist_host ? h->hst : nullptr, s));
            // The output goes out before the state is read: a solve that
            // needs no restart (nearly all) is then complete at the read.  A
            // restart pass scatters again.  (With the V_0 shift the output
            // waits for the last pass: the shift changes x.)
            if (!h->singular) {
                hipLaunchKernelGGL(k_scatter, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->x, p_dev);
                HIPCK(hipGetLastError());
            }
            if (hist_host) HIPCK(hipStreamSynchronize(s));
            else TRY(read_state(h, s));
        }
        for (; !small;) {
            const size_t t0 = timed;
            TRY(launch_iterations(h, k, chunk, first, &timed, s));
            const int kfirst = k;
            k += chunk;
            first = false;
            TRY(read_state(h, s));
            chunk = next_chunk(*h->hst, chunk, rr_seen, it_seen);
            rr_seen = h->hst->rr;
            it_seen = h->hst->iter;
            if (h->timing) {
                // sampled launches that ran a full iteration (k <= final count)
                size_t idx = t0;
                for (int kk = kfirst; kk < kfirst + (k - kfirst) && idx < timed; ++kk) {
                    if ((kk % TIMING_STRIDE) != 1) continue;
                    const bool full = !h->hst->done || kk <= h->hst->iter;
                    if (full) {
                        float ms = 0.f;
                        HIPCK(hipEventElapsedTime(&ms, h->ev[2 * idx], h->ev[2 * idx + 1]));
                        h->t_ms += ms;
                        h->t_launches++;
                    }
                    ++idx;
                }
            }
            if (h->hst->done) break;
        }
        if (h->hst->status != 0) break;
        if (!(h->hst->bnorm > 0.0)) break;
        // true residual of the final iterate (the one-launch pass formed it)
        const int kdone = h->hst->iter;
        if (!small) {
            TRY(launch_apply(h, h->x, h->q, nullptr, s));
            hipLaunchKernelGGL(k_true_residual, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->r,
                               h->part_rr(kdone & 1));
            hipLaunchKernelGGL(k_finish_tt, dim3(1), dim3(BLK), 0, s, h->st, h->part_rr(kdone & 1), int(vg));
            HIPCK(hipGetLastError());
            TRY(read_state(h, s));
        }
        const double rel = std::sqrt(h->hst->tt) / h->hst->bnorm;
        if (rel <= rtol || replaced >= 2 || kdone >= max_iter) break;
        // residual replacement: r is now the true residual; restart the directions
        hipLaunchKernelGGL(k_reopen, dim3(1), dim3(64), 0, s, h->st);
        HIPCK(hipGetLastError());
        k = kdone + 1;
        first = true;
        ++replaced;
    }
    TRY(shift_mean(h, s));
    if (!(small && !h->singular)) {
        hipLaunchKernelGGL(k_scatter, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->x, p_dev);
        HIPCK(hipGetLastError());
    }
    const CGState fin = *h->hst;
    if (res_hist && hist_host) std::memcpy(res_hist, hist_host, sizeof(double) * size_t(fin.iter + 1));
    else if (res_hist)
        HIPCK(hipMemcpyAsync(res_hist, h->hist, sizeof(double) * (fin.iter + 1), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    *iters = fin.iter;
    double rel = 0.0;
    if (fin.bnorm > 0.0) rel = std::sqrt(fin.tt) / fin.bnorm;
    if (true_relres) *true_relres = rel;
    if (fin.status != 0) return fin.status;
    return (rel <= rtol) ? PM_OK : PM_NOT_CONVERGED;
}

int pressure_solve_noalloc(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                           int32_t max_iter, double *p_dev, int32_t *iters, double *res_hist,
                           double *true_relres, void *stream)
{
    if (!h || max_iter < 0) return PM_EINVAL;
    if (h->N > PM_NOALLOC_MAX_NODES || max_iter > PM_NOALLOC_MAX_ITER) return PM_ETOOLARGE;
    double *base = noalloc_scratch(h->device);
    if (!base) return PM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    ScratchSwap swap(h, base);
    // the direction buffers start at zero, as the handle's own do after setup
    hipLaunchKernelGGL(k_fill2, dim3(grid_of(h->N)), dim3(BLK), 0, s, h->N, h->pbuf[0], h->pbuf[1], 0.0);
    HIPCK(hipGetLastError());
    return pressure_solve(h, rhs_dev, x0_dev, rtol, max_iter, p_dev, iters, res_hist, true_relres, stream);
}

// Launch FP32 inner-CG iterations k0 .. k0+count-1.
static int launch_iterations32(pm_handle *h, int k0, int count, bool first, hipStream_t s)
{
    const int N = int(h->N);
    for (int c = 0; c < count; ++c) {
        const int k = k0 + c;
        IterT<float> it;
        it.k = k;
        it.first = (first && c == 0) ? 1 : 0;
        it.r = h->r32;
        it.p_old = h->p32[(k - 1) & 1];
        it.p_new = h->p32[k & 1];
        it.q = h->q32;
        it.st = h->st_in;
        it.hist = h->hist;
        it.part_pq = h->part_pq();
        it.rr_cur = h->part_rr((k - 1) & 1);
        it.rr_prev = h->part_rr(k & 1);
        it.n_vblocks = h->n_vblocks;
        TRY(launch_apply32(h, it, s));
        hipLaunchKernelGGL(k_update<float>, dim3(h->n_vblocks), dim3(BLK), 0, s, N, h->d32, h->r32, h->p32[k & 1],
                           h->q32, h->st_in, h->part_pq(), h->n_ablocks32, h->part_rr((k - 1) & 1), h->n_vblocks,
                           h->part_rr(k & 1));
    }
    HIPCK(hipGetLastError());
    return PM_OK;
}

int pressure_solve_mixed(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                         double inner_rtol, int32_t max_iter, double *p_dev, int32_t *iters,
                         int32_t *outer, double *res_hist, double *true_relres, void *stream)
{
    constexpr int MAX_OUTER = 64;
    if (!h || !rhs_dev || !p_dev || !iters || !(rtol > 0.0) || !std::isfinite(rtol) || max_iter < 0 ||
        !(inner_rtol > 0.0) || !(inner_rtol < 1.0))
        return PM_EINVAL;
    if (!h->coords32) return PM_EINVAL;   // handle built without PM_FP32_INNER
    hipStream_t s = (hipStream_t)stream;
    TRY(ensure_hist(h, max_iter));
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;
    std::vector<double> hist;

    hipLaunchKernelGGL(k_prepare, dim3(vg), dim3(BLK), 0, s, N, h->new2old, h->dir, rhs_dev, x0_dev, h->b, h->x,
                       h->part_misc());
    TRY(project_rhs(h, s));
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg), rtol, max_iter, h->hist, 1);
    HIPCK(hipGetLastError());
    TRY(read_state(h, s));
    int status = h->hst->status;
    const double bnorm = h->hst->bnorm;
    int total = 0, n_outer = 0, k = 1;
    const bool keep = h->mixed_mode == PM_MIXED_KEEP_DIRECTION;
    double rel = 0.0;
    if (status == 0 && !(bnorm > 0.0)) {
        // zero right-hand side: p = 0
        HIPCK(hipMemsetAsync(h->x, 0, 8 * size_t(N), s));
        hist.push_back(0.0);
    }
    while (status == 0 && bnorm > 0.0) {
        // outer FP64 residual
        TRY(launch_apply(h, h->x, h->q, nullptr, s));
        hipLaunchKernelGGL(k_true_residual, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->r, h->part_misc());
        hipLaunchKernelGGL(k_finish_tt, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg));
        HIPCK(hipGetLastError());
        TRY(read_state(h, s));
        rel = std::sqrt(h->hst->tt) / bnorm;
        hist.push_back(rel);
        if (!std::isfinite(rel)) {
            status = PM_EBREAKDOWN;
            break;
        }
        if (rel <= rtol || total >= max_iter || n_outer >= MAX_OUTER) break;
        // inner FP32 CG on A32 d = r32 from d = 0: a fresh CG (restart mode,
        // and the first correction), or the running one with its residual
        // replaced by the rounded FP64 residual and its direction kept
        const bool resume = keep && n_outer > 0;
        if (!resume) k = 1;
        double *rr_next = h->part_rr((k - 1) & 1);   // r.r partials the next apply reads
        hipLaunchKernelGGL(k_to_inner, dim3(vg), dim3(BLK), 0, s, N, h->r, h->r32, h->d32, rr_next);
        if (resume)
            hipLaunchKernelGGL(k_resume_inner, dim3(1), dim3(BLK), 0, s, h->st_in, rr_next, int(vg), inner_rtol, 1);
        else
            hipLaunchKernelGGL(k_begin_inner, dim3(1), dim3(BLK), 0, s, h->st_in, rr_next, int(vg), inner_rtol,
                               keep ? max_iter : max_iter - total, 1);
        HIPCK(hipGetLastError());
        const int iter0 = resume ? h->hst_in->iter : 0;
        int chunk = 4;
        bool first = !resume;
        double rr_seen = -1.0;
        int it_seen = 0;
        for (;;) {
            TRY(launch_iterations32(h, k, chunk, first, s));
            k += chunk;
            first = false;
            HIPCK(hipMemcpyAsync(h->hst_in, h->st_in, sizeof(CGState), hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            if (h->hst_in->done) break;
            chunk = next_chunk(*h->hst_in, chunk, rr_seen, it_seen);
            rr_seen = h->hst_in->rr;
            it_seen = h->hst_in->iter;
        }
        const int done_iter = h->hst_in->iter;   // last completed inner iteration
        k = done_iter + 1;
        total = keep ? done_iter : total + done_iter;
        if (h->hst_in->status != 0) {
            status = h->hst_in->status;
            break;
        }
        // no inner progress (the rounded residual is zero, d = 0): x is final
        if (done_iter == iter0) break;
        hipLaunchKernelGGL(k_correct, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->x, h->d32);
        HIPCK(hipGetLastError());
        ++n_outer;
    }
    TRY(shift_mean(h, s));
    hipLaunchKernelGGL(k_scatter, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->x, p_dev);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    *iters = total;
    if (outer) *outer = n_outer;
    if (res_hist)
        for (size_t i = 0; i < hist.size() && i <= size_t(max_iter); ++i) res_hist[i] = hist[i];
    if (true_relres) *true_relres = rel;
    if (status != 0) return status;
    return (rel <= rtol) ? PM_OK : PM_NOT_CONVERGED;
}

int pressure_set_variant(pm_handle *h, int32_t variant)
{
    if (!h) return PM_EINVAL;
    switch (variant) {
    case PM_VARIANT_AUTO: h->variant = (h->tile_class >= 0) ? PM_VARIANT_TILED : PM_VARIANT_NODE; return PM_OK;
    case PM_VARIANT_TILED:
        if (h->tile_class < 0) return PM_EINVAL;   // mesh on the node kernel only
        h->variant = PM_VARIANT_TILED;
        return PM_OK;
    case PM_VARIANT_NODE: h->variant = PM_VARIANT_NODE; return PM_OK;
    default: return PM_EINVAL;
    }
}

int pressure_set_mixed_mode(pm_handle *h, int32_t mode)
{
    if (!h || (mode != PM_MIXED_KEEP_DIRECTION && mode != PM_MIXED_RESTART)) return PM_EINVAL;
    h->mixed_mode = mode;
    return PM_OK;
}

int pressure_timing_enable(pm_handle *h, int32_t enable)
{
    if (!h) return PM_EINVAL;
    h->timing = enable != 0;
    h->t_launches = 0;
    h->t_ms = 0.0;
    return PM_OK;
}

int pressure_timing_read(pm_handle *h, int64_t *launches, double *total_ms)
{
    if (!h || !launches || !total_ms) return PM_EINVAL;
    *launches = h->t_launches;
    *total_ms = h->t_ms;
    return PM_OK;
}

int pressure_info(pm_handle *h, int64_t *info, int32_t n_info)
{
    if (!h || !info || n_info < 0) return PM_EINVAL;
    const int64_t d = h->dim;
    int64_t v[9] = {h->N, h->E, h->n_free, d,
                    16 * h->N + 8 * d * h->N + 4 * (d + 1) * h->E + 8 * h->E,
                    int64_t(h->dev_bytes), h->n_tiles, h->n_inst, small_ok(h) ? 1 : 0};
    for (int k = 0; k < n_info && k < 9; ++k) info[k] = v[k];
    return PM_OK;
}

}  // extern "C"

// ======================================================================
// Batched solves

struct pm_batch {
    std::vector<pm_handle *> hs;
    int device = 0;
    bool mixed = false;            // FP32 inner solves with FP64 corrections
    bool periodic = false;         // some mesh is periodic: the apply takes minimum images
    double inner_rtol = 1e-2;
    int tiles_per_slot = 4, nodes_per_lane = 8;
    void *d_meshes = nullptr;      // BatchMeshT<double> or BatchMeshT<float>
    int2 *d_aslots = nullptr, *d_uslots = nullptr;
    int n_aslots = 0, n_uslots = 0;
    // continuous batching: the slots of the meshes in flight (begun and not
    // yet finished), so that a step launches no blocks for idle meshes
    std::vector<int> a_off, u_off;          // per mesh: first apply / update slot (n + 1 entries)
    std::vector<uint8_t> in_flight;         // per mesh
    int2 *d_aslots_act = nullptr, *d_uslots_act = nullptr;
    int2 *h_slots_act = nullptr;            // pinned staging of both active tables
    int n_aslots_act = 0, n_uslots_act = 0;
    bool act_dirty = true;
    BatchCtl *d_ctl = nullptr, *h_ctl = nullptr;
    GridBar *d_bar = nullptr;          // persistent launches: grid barrier state (zeroed)
    CGState *d_states = nullptr, *h_states = nullptr;
    int bclass = -1;
    size_t lds = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t pgraph = nullptr;       // persistent form: its launch over every slot, captured
    hipGraphExec_t pgexec = nullptr;
    bool pgraph_failed = false;        // the runtime would not capture it: launch directly
    int graph_iters = 16;
    bool persistent = false;           // one cooperative launch per step (k_batch_persistent)
    bool step_pending = false;         // pressure_batch_step_launch without its _wait yet
    int coop_grid = 0;                 // resident blocks of the persistent kernel (0: not yet known)
    long long bar_limit = 200000000;   // grid barrier time limit, 100 MHz ticks (2 s)
    int k_next = 1;          // launch index of the next batched iteration
    std::vector<double *> hist_seen;   // history pointers in the uploaded descriptors
};

namespace {

enum { MX_IDLE = 0, MX_RESIDUAL = 1, MX_INNER = 2, MX_FINISHED = 3 };
constexpr int MAX_CORRECTIONS = 64;

// The batched apply runs the size classes of 128-node tiles (the first
// N_BATCH_CLASSES entries of TILE_CLASSES).
constexpr int N_BATCH_CLASSES = 6;
static_assert(TILE_CLASSES[N_BATCH_CLASSES - 1].t == 128 && TILE_CLASSES[N_BATCH_CLASSES].t != 128 &&
                  TILE_CLASSES[N_BATCH_CLASSES - 1].nth == BLK,
              "batch classes are the 128-node classes");

// A batch with a periodic mesh runs the minimum-image kernels for all its
// meshes (exact no-ops on the open axes, so the other meshes get the same
// bits as alone).
template <class R, bool PER>
const void *batch_apply_kernel(int c)
{
    switch (c) {
    case 0: return (const void *)k_batch_apply<0, R, PER>;
    case 1: return (const void *)k_batch_apply<1, R, PER>;
    case 2: return (const void *)k_batch_apply<2, R, PER>;
    case 3: return (const void *)k_batch_apply<3, R, PER>;
    case 4: return (const void *)k_batch_apply<4, R, PER>;
    case 5: return (const void *)k_batch_apply<5, R, PER>;
    default: return nullptr;
    }
}

template <class R>
const void *batch_apply_kernel(const pm_batch *b)
{
    return b->periodic ? batch_apply_kernel<R, true>(b->bclass) : batch_apply_kernel<R, false>(b->bclass);
}

template <int C, class R>
void launch_batch_apply_c(pm_batch *b, const int2 *slots, int n_slots, hipStream_t s)
{
    if (b->periodic)
        hipLaunchKernelGGL((k_batch_apply<C, R, true>), dim3(n_slots), dim3(BLK), b->lds, s,
                           (const BatchMeshT<R> *)b->d_meshes, slots, b->d_ctl);
    else
        hipLaunchKernelGGL((k_batch_apply<C, R, false>), dim3(n_slots), dim3(BLK), b->lds, s,
                           (const BatchMeshT<R> *)b->d_meshes, slots, b->d_ctl);
}

// count iterations over the slots of every mesh (active = false: the
// captured graph) or of the meshes in flight only (the active tables).
template <class R>
int launch_batch_iterations_t(pm_batch *b, int count, bool active, hipStream_t s)
{
    const int2 *as = active ? b->d_aslots_act : b->d_aslots;
    const int2 *us = active ? b->d_uslots_act : b->d_uslots;
    const int na = active ? b->n_aslots_act : b->n_aslots, nu = active ? b->n_uslots_act : b->n_uslots;
    for (int i = 0; i < count; ++i) {
        switch (b->bclass) {
        case 0: launch_batch_apply_c<0, R>(b, as, na, s); break;
        case 1: launch_batch_apply_c<1, R>(b, as, na, s); break;
        case 2: launch_batch_apply_c<2, R>(b, as, na, s); break;
        case 3: launch_batch_apply_c<3, R>(b, as, na, s); break;
        case 4: launch_batch_apply_c<4, R>(b, as, na, s); break;
        case 5: launch_batch_apply_c<5, R>(b, as, na, s); break;
        default: return PM_EINVAL;
        }
        hipLaunchKernelGGL(k_batch_update<R>, dim3(nu), dim3(BLK), 0, s, (const BatchMeshT<R> *)b->d_meshes, us,
                           b->d_ctl);
    }
    HIPCK(hipGetLastError());
    return PM_OK;
}

int launch_batch_iterations(pm_batch *b, int count, bool active, hipStream_t s)
{
    return b->mixed ? launch_batch_iterations_t<float>(b, count, active, s)
                    : launch_batch_iterations_t<double>(b, count, active, s);
}

template <class R, bool PER>
const void *batch_persistent_kernel(int c)
{
    switch (c) {
    case 0: return (const void *)k_batch_persistent<0, R, PER>;
    case 1: return (const void *)k_batch_persistent<1, R, PER>;
    case 2: return (const void *)k_batch_persistent<2, R, PER>;
    case 3: return (const void *)k_batch_persistent<3, R, PER>;
    case 4: return (const void *)k_batch_persistent<4, R, PER>;
    case 5: return (const void *)k_batch_persistent<5, R, PER>;
    default: return nullptr;
    }
}

// count iterations of the meshes in flight as one cooperative launch of
// the persistent kernel, with as many blocks as can be resident (at most
// one per slot).  The runtime rejects a cooperative grid that cannot be
// resident at once.
template <class R>
int launch_batch_persistent_t(pm_batch *b, int count, bool active, hipStream_t s)
{
    const void *kern = b->periodic ? batch_persistent_kernel<R, true>(b->bclass)
                                   : batch_persistent_kernel<R, false>(b->bclass);
    if (!kern) return PM_EINVAL;
    if (b->coop_grid <= 0) {
        int per_cu = 0, cus = 0;
        HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLK, b->lds));
        HIPCK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        if (per_cu < 1 || cus < 1) return PM_EHIP;
        b->coop_grid = per_cu * cus;
    }
    const BatchMeshT<R> *meshes = (const BatchMeshT<R> *)b->d_meshes;
    const int2 *as = active ? b->d_aslots_act : b->d_aslots, *us = active ? b->d_uslots_act : b->d_uslots;
    int na = active ? b->n_aslots_act : b->n_aslots, nu = active ? b->n_uslots_act : b->n_uslots;
    const int grid = std::min(b->coop_grid, std::max(na, nu));
    if (grid < 1 || count < 1) return PM_OK;
    BatchCtl *ctl = b->d_ctl;
    GridBar *gb = b->d_bar;
    long long limit = b->bar_limit;
    void *args[] = {(void *)&meshes, (void *)&as, (void *)&na, (void *)&us, (void *)&nu, (void *)&ctl,
                    (void *)&gb, (void *)&count, (void *)&limit};
    HIPCK(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(BLK), args, (unsigned)b->lds, s));
    return PM_OK;
}

int launch_batch_persistent(pm_batch *b, int count, bool active, hipStream_t s)
{
    return b->mixed ? launch_batch_persistent_t<float>(b, count, active, s)
                    : launch_batch_persistent_t<double>(b, count, active, s);
}

void drop_graph(hipGraph_t *g, hipGraphExec_t *e)
{
    if (*e) (void)hipGraphExecDestroy(*e);
    if (*g) (void)hipGraphDestroy(*g);
    *e = nullptr;
    *g = nullptr;
}

// The persistent form's step over every slot, captured once in a HIP graph
// (a cooperative kernel node).  If the runtime will not capture the
// cooperative launch, the step launches it directly from then on.
int batch_capture_persistent(pm_batch *b)
{
    drop_graph(&b->pgraph, &b->pgexec);
    // the resident-block count is queried before the capture (no launch: count 0)
    TRY(launch_batch_persistent(b, 0, false, b->stream));
    HIPCK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int st = launch_batch_persistent(b, b->graph_iters, false, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    (void)hipGetLastError();
    if (st != PM_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        b->pgraph_failed = true;
        if (std::getenv("PM_DEBUG"))
            std::fprintf(stderr, "libpressure: persistent batch launch not captured (%s); launching directly\n",
                         hipGetErrorString(e));
        return PM_OK;
    }
    if (std::getenv("PM_DEBUG")) std::fprintf(stderr, "libpressure: persistent batch launch captured in a graph\n");
    b->pgraph = g;
    if (hipGraphInstantiate(&b->pgexec, b->pgraph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        drop_graph(&b->pgraph, &b->pgexec);
        b->pgraph_failed = true;
    }
    return PM_OK;
}

// Upload the slot tables of the meshes in flight (in mesh order, each
// mesh's slots in order), in stream order.
int refresh_active_slots(pm_batch *b, hipStream_t s)
{
    if (!b->act_dirty) return PM_OK;
    // the staging buffer is free: every step ends with its stream synchronised
    const int n = int(b->hs.size());
    int na = 0, nu = 0;
    int2 *ha = b->h_slots_act, *hu = b->h_slots_act + b->n_aslots;
    for (int m = 0; m < n; ++m) {
        if (!b->in_flight[m]) continue;
        for (int j = b->a_off[m]; j < b->a_off[m + 1]; ++j) ha[na++] = make_int2(m, j - b->a_off[m]);
        for (int j = b->u_off[m]; j < b->u_off[m + 1]; ++j) hu[nu++] = make_int2(m, j - b->u_off[m]);
    }
    if (na > 0) HIPCK(hipMemcpyAsync(b->d_aslots_act, ha, sizeof(int2) * na, hipMemcpyHostToDevice, s));
    if (nu > 0) HIPCK(hipMemcpyAsync(b->d_uslots_act, hu, sizeof(int2) * nu, hipMemcpyHostToDevice, s));
    b->n_aslots_act = na;
    b->n_uslots_act = nu;
    b->act_dirty = false;
    return PM_OK;
}

void batch_free(pm_batch *b)
{
    if (!b) return;
    // work queued by begin / finish completes first: a batch rebuilt over
    // the same handles reads their solver states
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    drop_graph(&b->pgraph, &b->pgexec);
    for (void *p : {(void *)b->d_meshes, (void *)b->d_aslots, (void *)b->d_uslots, (void *)b->d_ctl, (void *)b->d_bar,
                    (void *)b->d_states, (void *)b->d_aslots_act, (void *)b->d_uslots_act})
        if (p) (void)hipFree(p);
    if (b->h_slots_act) (void)hipHostFree(b->h_slots_act);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    if (b->h_states) (void)hipHostFree(b->h_states);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Descriptor of one mesh of the batch: its FP64 solve, or (mixed) its FP32
// inner solve.
template <class R>
BatchMeshT<R> batch_mesh(pm_handle *h);

template <>
BatchMeshT<double> batch_mesh<double>(pm_handle *h)
{
    BatchMeshT<double> M;
    M.dim = h->dim;
    M.N = int(h->N);
    M.g = make_mesh<double>(h);
    M.ta = make_tiles<double>(h);
    M.x = h->x;
    M.r = h->r;
    M.q = h->q;
    M.p0 = h->pbuf[0];
    M.p1 = h->pbuf[1];
    M.hist = h->hist;
    M.st = h->st;
    M.part_pq = h->part_pq();
    M.rr0 = h->part_rr(0);
    M.rr1 = h->part_rr(1);
    M.n_ab = h->n_ablocks;
    M.n_vb = h->n_vblocks;
    return M;
}

template <>
BatchMeshT<float> batch_mesh<float>(pm_handle *h)
{
    BatchMeshT<float> M;
    M.dim = h->dim;
    M.N = int(h->N);
    M.g = make_mesh<float>(h);
    M.ta = make_tiles<float>(h);
    M.x = h->d32;
    M.r = h->r32;
    M.q = h->q32;
    M.p0 = h->p32[0];
    M.p1 = h->p32[1];
    M.hist = h->hist;
    M.st = h->st_in;
    M.part_pq = h->part_pq();
    M.rr0 = h->part_rr(0);
    M.rr1 = h->part_rr(1);
    M.n_ab = h->n_ablocks32;
    M.n_vb = h->n_vblocks;
    return M;
}

template <class R>
int upload_meshes(pm_batch *b)
{
    std::vector<BatchMeshT<R>> meshes;
    b->hist_seen.clear();
    for (pm_handle *h : b->hs) {
        meshes.push_back(batch_mesh<R>(h));
        b->hist_seen.push_back(h->hist);
    }
    if (!b->d_meshes && hipMalloc(&b->d_meshes, sizeof(BatchMeshT<R>) * meshes.size()) != hipSuccess)
        return PM_ENOMEM;
    HIPCK(hipMemcpyAsync(b->d_meshes, meshes.data(), sizeof(BatchMeshT<R>) * meshes.size(), hipMemcpyHostToDevice,
                         b->stream));
    HIPCK(hipStreamSynchronize(b->stream));
    return PM_OK;
}

int batch_create_impl(pm_batch *b, pm_handle *const *handles, int32_t n, const int32_t *params)
{
    int k_start = 1;
    if (params) {
        if (params[0] < 1 || params[1] < 1 || params[2] < 1) return PM_EINVAL;
        b->tiles_per_slot = params[0];
        b->nodes_per_lane = params[1];
        k_start = params[2];
    }
    HIPCK(hipGetDevice(&b->device));
    int max_inst = 1, max_local = 1;
    std::vector<int2> aslots, uslots;
    for (int m = 0; m < n; ++m) {
        pm_handle *h = handles[m];
        if (!h || h->device != b->device || h->tile_class < 0 || TILE_CLASSES[h->tile_class].t != 128)
            return PM_EINVAL;
        if (b->mixed && !h->coords32) return PM_EINVAL;   // handle built without PM_FP32_INNER
        max_inst = std::max(max_inst, h->max_inst);
        max_local = std::max(max_local, h->max_local);
        b->periodic = b->periodic || h->periodic;
        // the batch's grids become the handle's
        h->n_ablocks = std::max(1, std::min(AGRID_MAX, (h->n_tiles + b->tiles_per_slot - 1) / b->tiles_per_slot));
        h->n_ablocks32 = h->n_ablocks;
        h->n_vblocks = int(std::max<int64_t>(1, std::min<int64_t>(VGRID_MAX, (h->N + int64_t(BLK) * b->nodes_per_lane - 1) /
                                                                                 (int64_t(BLK) * b->nodes_per_lane))));
        b->a_off.push_back(int(aslots.size()));
        b->u_off.push_back(int(uslots.size()));
        for (int j = 0; j < h->n_ablocks; ++j) aslots.push_back(make_int2(m, j));
        for (int j = 0; j < h->n_vblocks; ++j) uslots.push_back(make_int2(m, j));
        b->hs.push_back(h);
    }
    b->bclass = -1;
    for (int c = 0; c < N_BATCH_CLASSES; ++c)
        if (TILE_CLASSES[c].ipt * BLK >= max_inst && TILE_CLASSES[c].lm >= max_local) {
            b->bclass = c;
            break;
        }
    if (b->bclass < 0) return PM_EINVAL;
    for (pm_handle *h : b->hs)
        b->lds = std::max(b->lds, b->mixed ? tiled_lds_bytes<float>(h->dim, b->bclass, h->max_deg)
                                           : tiled_lds_bytes<double>(h->dim, b->bclass, h->max_deg));
    if (b->lds > b->hs[0]->lds_limit) return PM_EINVAL;
    if (b->lds > 65536) {
        const void *k = b->mixed ? batch_apply_kernel<float>(b) : batch_apply_kernel<double>(b);
        HIPCK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(b->lds)));
    }
    b->n_aslots = int(aslots.size());
    b->n_uslots = int(uslots.size());
    auto up = [&](auto **dst, const auto &vec) -> int {
        using T = typename std::remove_reference<decltype(vec)>::type::value_type;
        if (hipMalloc((void **)dst, sizeof(T) * vec.size()) != hipSuccess) return PM_ENOMEM;
        HIPCK(hipMemcpy(*dst, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice));
        return PM_OK;
    };
    TRY(up(&b->d_aslots, aslots));
    TRY(up(&b->d_uslots, uslots));
    b->a_off.push_back(b->n_aslots);
    b->u_off.push_back(b->n_uslots);
    b->in_flight.assign(n, 0);
    TRY(up(&b->d_aslots_act, aslots));
    TRY(up(&b->d_uslots_act, uslots));
    HIPCK(hipHostMalloc((void **)&b->h_slots_act, sizeof(int2) * (b->n_aslots + b->n_uslots), hipHostMallocDefault));
    if (hipMalloc((void **)&b->d_ctl, sizeof(BatchCtl)) != hipSuccess) return PM_ENOMEM;
    if (hipMalloc((void **)&b->d_bar, sizeof(GridBar)) != hipSuccess) return PM_ENOMEM;
    HIPCK(hipMemset(b->d_bar, 0, sizeof(GridBar)));
    if (hipMalloc((void **)&b->d_states, sizeof(CGState) * n) != hipSuccess) return PM_ENOMEM;
    HIPCK(hipHostMalloc((void **)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault));
    HIPCK(hipHostMalloc((void **)&b->h_states, sizeof(CGState) * n, hipHostMallocDefault));
    std::memset(b->h_states, 0, sizeof(CGState) * n);   // no inner solve is seen as stopped before a step
    HIPCK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIPCK(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
    TRY(b->mixed ? upload_meshes<float>(b) : upload_meshes<double>(b));
    // a batch rebuilt over handles whose solves are running (begun in an
    // earlier batch, not finished) continues them: they are in flight here
    for (int m = 0; m < n; ++m) {
        pm_handle *h = b->hs[m];
        if (b->mixed) {
            b->in_flight[m] = (h->mx.phase == MX_RESIDUAL || h->mx.phase == MX_INNER) ? 1 : 0;
        } else {
            CGState st{};
            HIPCK(hipMemcpy(&st, h->st, sizeof(CGState), hipMemcpyDeviceToHost));
            b->in_flight[m] = st.done ? 0 : 1;
        }
    }
    b->act_dirty = true;
    // solves of the handles that are in flight continue at launch index k_start
    b->k_next = k_start;
    std::memset(b->h_ctl, 0, sizeof(BatchCtl));
    b->h_ctl->k_apply = k_start;
    b->h_ctl->k_update = k_start - 1;
    b->h_ctl->n_done = 0;
    HIPCK(hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, b->stream));
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(b->stream));
    return PM_OK;
}

int batch_capture(pm_batch *b)
{
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (b->graph_iters <= 0) return PM_OK;
    HIPCK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int st = launch_batch_iterations(b, b->graph_iters, false, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != PM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCK(e);
    b->graph = g;
    HIPCK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    return PM_OK;
}

int batch_create_common(pm_handle *const *handles, int32_t n, const int32_t *params, bool mixed, double inner_rtol,
                        pm_batch **out)
{
    if (!out || !handles || n < 1) return PM_EINVAL;
    *out = nullptr;
    pm_batch *b = nullptr;
    try {
        b = new pm_batch();
        b->mixed = mixed;
        b->inner_rtol = inner_rtol;
        int s = batch_create_impl(b, handles, n, params);
        // the graph is captured at the first step that replays it
        if (s != PM_OK) {
            batch_free(b);
            return s;
        }
    } catch (...) {
        batch_free(b);
        return PM_ENOMEM;
    }
    *out = b;
    return PM_OK;
}

// The histories may have been reallocated (ensure_hist): refresh descriptors.
int batch_refresh(pm_batch *b)
{
    bool moved = false;
    for (size_t m = 0; m < b->hs.size(); ++m) moved |= (b->hs[m]->hist != b->hist_seen[m]);
    if (!moved) return PM_OK;
    return b->mixed ? upload_meshes<float>(b) : upload_meshes<double>(b);
}

// Start the FP64 solve of mesh m at the batch's next launch index: gather rhs
// and guess, ||rhs||, r0 = rhs - A x0 (partials into the buffer its first
// apply reads).  A mixed solve only gathers here; its FP64 residual is
// computed by the next step's correction pass.
int batch_begin_impl(pm_batch *b, int m, const double *rhs_dev, const double *x0_dev, double rtol,
                     int32_t max_iter, hipStream_t s)
{
    pm_handle *h = b->hs[m];
    TRY(ensure_hist(h, max_iter));
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;
    if (!b->in_flight[m]) {
        b->in_flight[m] = 1;
        b->act_dirty = true;
    }
    hipLaunchKernelGGL(k_prepare, dim3(vg), dim3(BLK), 0, s, N, h->new2old, h->dir, rhs_dev, x0_dev, h->b, h->x,
                       h->part_misc());
    TRY(project_rhs(h, s));
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg), rtol, max_iter, h->hist,
                       b->k_next);
    if (b->mixed) {
        pm_handle::MixedSolve &X = b->hs[m]->mx;
        X = pm_handle::MixedSolve();
        X.phase = MX_RESIDUAL;
        X.rtol = rtol;
        X.max_iter = max_iter;
        HIPCK(hipGetLastError());
        return PM_OK;
    }
    TRY(launch_apply(h, h->x, h->q, nullptr, s));
    hipLaunchKernelGGL(k_start, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->x, h->r, h->st, h->part_rr(0));
    HIPCK(hipGetLastError());
    return PM_OK;
}

// Mixed batches: FP64 residual r = b - A x for every mesh whose inner solve
// has stopped (after x += d) or that has just begun, then the decision per
// mesh: finished, or (re)start its inner solve at the next launch.
int batch_corrections(pm_batch *b, hipStream_t s)
{
    const int n = int(b->hs.size());
    std::vector<int> due;
    for (int m = 0; m < n; ++m) {
        pm_handle::MixedSolve &X = b->hs[m]->mx;
        if (X.phase == MX_RESIDUAL) due.push_back(m);
        else if (X.phase == MX_INNER && b->h_states[m].done) due.push_back(m);
    }
    if (due.empty()) return PM_OK;
    for (int m : due) {
        pm_handle *h = b->hs[m];
        pm_handle::MixedSolve &X = b->hs[m]->mx;
        const int N = int(h->N);
        const unsigned vg = h->n_vblocks;
        if (X.phase == MX_INNER) {
            const CGState &in = b->h_states[m];
            const bool keep = h->mixed_mode == PM_MIXED_KEEP_DIRECTION;
            X.iters = keep ? in.iter : X.iters + in.iter;
            if (in.status != 0) {
                X.status = in.status;
                X.phase = MX_FINISHED;
                continue;
            }
            if (in.iter == X.iter0) {   // no inner progress: x is final
                X.phase = MX_FINISHED;
                continue;
            }
            hipLaunchKernelGGL(k_correct, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->x, h->d32);
            ++X.n_outer;
        }
        TRY(launch_apply(h, h->x, h->q, nullptr, s));
        hipLaunchKernelGGL(k_true_residual, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->r, h->part_misc());
        hipLaunchKernelGGL(k_finish_tt, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg));
        HIPCK(hipMemcpyAsync(h->hst, h->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    }
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    for (int m : due) {
        pm_handle *h = b->hs[m];
        pm_handle::MixedSolve &X = b->hs[m]->mx;
        if (X.phase == MX_FINISHED) continue;
        const int N = int(h->N);
        const unsigned vg = h->n_vblocks;
        const CGState &st = *h->hst;
        if (st.status != 0) {   // not finite rhs
            X.status = st.status;
            X.phase = MX_FINISHED;
            continue;
        }
        if (!(st.bnorm > 0.0)) {   // zero right-hand side: p = 0
            HIPCK(hipMemsetAsync(h->x, 0, 8 * size_t(N), s));
            X.rel = 0.0;
            X.phase = MX_FINISHED;
            continue;
        }
        X.rel = std::sqrt(st.tt) / st.bnorm;
        if (!std::isfinite(X.rel)) {
            X.status = PM_EBREAKDOWN;
            X.phase = MX_FINISHED;
            continue;
        }
        if (X.rel <= X.rtol || X.iters >= X.max_iter || X.n_outer >= MAX_CORRECTIONS) {
            X.phase = MX_FINISHED;
            continue;
        }
        const bool keep = h->mixed_mode == PM_MIXED_KEEP_DIRECTION;
        const bool resume = keep && X.phase == MX_INNER;
        const int K = resume ? b->h_states[m].iter : 0;   // last completed inner iteration
        double *rr_next = h->part_rr(K & 1);              // r.r partials of iteration K+1's apply
        hipLaunchKernelGGL(k_to_inner, dim3(vg), dim3(BLK), 0, s, N, h->r, h->r32, h->d32, rr_next);
        if (resume)
            hipLaunchKernelGGL(k_resume_inner, dim3(1), dim3(BLK), 0, s, h->st_in, rr_next, int(vg), b->inner_rtol,
                               b->k_next - K);
        else
            hipLaunchKernelGGL(k_begin_inner, dim3(1), dim3(BLK), 0, s, h->st_in, rr_next, int(vg), b->inner_rtol,
                               keep ? X.max_iter : X.max_iter - X.iters, b->k_next);
        X.iter0 = K;
        X.phase = MX_INNER;
    }
    HIPCK(hipGetLastError());
    return PM_OK;
}

bool batch_mesh_done(const pm_batch *b, int m)
{
    if (b->mixed) return b->hs[m]->mx.phase == MX_IDLE || b->hs[m]->mx.phase == MX_FINISHED;
    return b->h_states[m].done != 0;
}

// Advance every solve in flight by one chunk of iterations (mixed batches:
// after the correction pass); copies the states to b->h_states.
int batch_step_launch(pm_batch *b, hipStream_t s)
{
    const int n = int(b->hs.size());
    if (b->mixed) TRY(batch_corrections(b, s));
    TRY(refresh_active_slots(b, s));
    int its = 0;
    if (b->persistent) {
        // one cooperative launch over the slots of the meshes in flight;
        // with every mesh in flight, replayed from its captured graph
        its = b->graph_iters > 0 ? b->graph_iters : 8;
        if (b->graph_iters > 0 && b->n_aslots_act == b->n_aslots && !b->pgraph_failed) {
            if (!b->pgexec) TRY(batch_capture_persistent(b));
        }
        if (b->graph_iters > 0 && b->n_aslots_act == b->n_aslots && b->pgexec)
            HIPCK(hipGraphLaunch(b->pgexec, s));
        else if (b->n_aslots_act > 0)
            TRY(launch_batch_persistent(b, its, true, s));
        else
            its = 0;
    } else if (b->graph_iters > 0 && b->n_aslots_act == b->n_aslots) {
        // every mesh in flight: the captured graph over all slots (captured
        // on the batch's stream at the first such step)
        if (!b->gexec) TRY(batch_capture(b));
        HIPCK(hipGraphLaunch(b->gexec, s));
        its = b->graph_iters;
    } else if (b->n_aslots_act > 0) {
        // some meshes idle: launches over the slots of the meshes in flight
        its = b->graph_iters > 0 ? b->graph_iters : 8;
        TRY(launch_batch_iterations(b, its, true, s));
    }
    b->k_next += its;
    if (b->mixed)
        hipLaunchKernelGGL(k_batch_status<float>, dim3(1), dim3(BLK), 0, s, (const BatchMeshT<float> *)b->d_meshes, n,
                           b->d_ctl, b->d_states);
    else
        hipLaunchKernelGGL(k_batch_status<double>, dim3(1), dim3(BLK), 0, s, (const BatchMeshT<double> *)b->d_meshes,
                           n, b->d_ctl, b->d_states);
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(b->h_ctl, b->d_ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(b->h_states, b->d_states, sizeof(CGState) * n, hipMemcpyDeviceToHost, s));
    return PM_OK;
}

// The end of a step started by batch_step_launch: wait for it; the states
// are then in b->h_states.
int batch_step_wait(pm_batch *b, hipStream_t s)
{
    const int n = int(b->hs.size());
    HIPCK(hipStreamSynchronize(s));
    if (b->h_ctl->failed) {
        // a grid barrier timed out: the solves in flight are lost; clear the
        // barrier so the batch can be destroyed or its meshes begun again
        b->h_ctl->failed = 0;
        HIPCK(hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, s));
        HIPCK(hipMemsetAsync(b->d_bar, 0, sizeof(GridBar), s));
        HIPCK(hipStreamSynchronize(s));
        return PM_ETIMEOUT;
    }
    // solves that have stopped leave the active tables: later steps launch
    // no blocks for them (pressure_batch_finish still takes them)
    for (int m = 0; m < n; ++m)
        if (b->in_flight[m] && batch_mesh_done(b, m)) {
            b->in_flight[m] = 0;
            b->act_dirty = true;
        }
    return PM_OK;
}

int batch_step_impl(pm_batch *b, hipStream_t s)
{
    TRY(batch_step_launch(b, s));
    return batch_step_wait(b, s);
}


// True residual and output of a finished mesh; for FP64 solves, residual
// replacement (as in pressure_solve) when the recursive residual met rtol
// but the true one did not.
int batch_finish_impl(pm_batch *b, int m, const double *rhs_dev, double rtol, double *p_dev, int32_t *iters,
                      double *true_relres, hipStream_t s)
{
    pm_handle *h = b->hs[m];
    const int N = int(h->N);
    const unsigned vg = h->n_vblocks;
    if (b->in_flight[m]) {
        b->in_flight[m] = 0;
        b->act_dirty = true;
    }
    if (b->mixed) {
        pm_handle::MixedSolve &X = b->hs[m]->mx;
        TRY(shift_mean(h, s));
        hipLaunchKernelGGL(k_scatter, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->x, p_dev);
        HIPCK(hipGetLastError());
        HIPCK(hipStreamSynchronize(s));
        *iters = X.iters;
        *true_relres = X.rel;
        X.phase = MX_IDLE;
        if (X.status != 0) return X.status;
        return (X.rel <= rtol) ? PM_OK : PM_NOT_CONVERGED;
    }
    TRY(launch_apply(h, h->x, h->q, nullptr, s));
    hipLaunchKernelGGL(k_true_residual, dim3(vg), dim3(BLK), 0, s, N, h->b, h->q, h->r, h->part_misc());
    hipLaunchKernelGGL(k_finish_tt, dim3(1), dim3(BLK), 0, s, h->st, h->part_misc(), int(vg));
    TRY(shift_mean(h, s));
    hipLaunchKernelGGL(k_scatter, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->x, p_dev);
    HIPCK(hipGetLastError());
    TRY(read_state(h, s));
    const CGState st = *h->hst;
    *iters = st.iter;
    const double rel = (st.bnorm > 0.0) ? std::sqrt(st.tt) / st.bnorm : 0.0;
    *true_relres = rel;
    int code = st.status;
    if (code == 0 && !(rel <= rtol)) {
        if (st.iter >= st.max_iter) return PM_NOT_CONVERGED;
        int32_t more = 0;
        double rel2 = rel;
        code = pressure_solve(h, rhs_dev, p_dev, rtol, std::max(0, st.max_iter - st.iter), p_dev, &more, nullptr,
                              &rel2, (void *)s);
        *iters += more;
        *true_relres = rel2;
        // the handle is idle again for the batch
        hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, s, h->st);
        HIPCK(hipGetLastError());
    }
    return code;
}

}  // namespace

extern "C" {

int pressure_batch_create(pm_handle *const *handles, int32_t n, const int32_t *params, pm_batch **out)
{
    return batch_create_common(handles, n, params, false, 0.0, out);
}

int pressure_batch_create_mixed(pm_handle *const *handles, int32_t n, const int32_t *params, double inner_rtol,
                                pm_batch **out)
{
    if (!(inner_rtol > 0.0) || !(inner_rtol < 1.0)) return PM_EINVAL;
    return batch_create_common(handles, n, params, true, inner_rtol, out);
}

void pressure_batch_destroy(pm_batch *b) { batch_free(b); }

int pressure_batch_set_graph(pm_batch *b, int32_t iterations_per_replay)
{
    if (!b || iterations_per_replay < 0 || iterations_per_replay > 256 || (iterations_per_replay % 2) != 0)
        return PM_EINVAL;
    b->graph_iters = iterations_per_replay;
    drop_graph(&b->pgraph, &b->pgexec);
    // the graph of the new length is captured at the next step that replays it
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    return PM_OK;
}

int pressure_batch_set_persistent(pm_batch *b, int32_t persistent)
{
    if (!b || (persistent != 0 && persistent != 1)) return PM_EINVAL;
    b->persistent = persistent != 0;
    drop_graph(&b->pgraph, &b->pgexec);
    return PM_OK;
}

int pressure_batch_set_barrier_limit(pm_batch *b, int64_t microseconds)
{
    if (!b || microseconds < 0 || microseconds > int64_t(600) * 1000000) return PM_EINVAL;
    b->bar_limit = (microseconds == 0) ? 200000000LL : 100LL * microseconds;   // 100 MHz ticks
    drop_graph(&b->pgraph, &b->pgexec);   // the captured launch holds the old limit
    return PM_OK;
}

int pressure_batch_begin(pm_batch *b, int32_t m, const double *rhs_dev, const double *x0_dev, double rtol,
                         int32_t max_iter, void *stream)
{
    if (!b || b->step_pending || m < 0 || m >= int(b->hs.size()) || !rhs_dev || !(rtol > 0.0) || !std::isfinite(rtol) || max_iter < 0)
        return PM_EINVAL;
    hipStream_t us = (hipStream_t)stream, s = b->stream;
    HIPCK(hipEventRecord(b->ev, us));
    HIPCK(hipStreamWaitEvent(s, b->ev, 0));
    TRY(batch_begin_impl(b, m, rhs_dev, x0_dev, rtol, max_iter, s));
    return batch_refresh(b);
}

int pressure_batch_step_launch(pm_batch *b, void *stream)
{
    if (!b || b->step_pending) return PM_EINVAL;
    HIPCK(hipEventRecord(b->ev, (hipStream_t)stream));
    HIPCK(hipStreamWaitEvent(b->stream, b->ev, 0));
    TRY(batch_step_launch(b, b->stream));
    b->step_pending = true;
    return PM_OK;
}

int pressure_batch_step_poll(pm_batch *b, int32_t *done)
{
    if (!b || !done || !b->step_pending) return PM_EINVAL;
    const hipError_t q = hipStreamQuery(b->stream);
    if (q == hipErrorNotReady) return PM_PENDING;
    if (q != hipSuccess) return hip_failed(q, "hipStreamQuery(b->stream)", __LINE__);
    return pressure_batch_step_wait(b, done);
}

int pressure_batch_step_wait(pm_batch *b, int32_t *done)
{
    if (!b || !done || !b->step_pending) return PM_EINVAL;
    b->step_pending = false;
    TRY(batch_step_wait(b, b->stream));
    for (size_t m = 0; m < b->hs.size(); ++m) done[m] = batch_mesh_done(b, int(m)) ? 1 : 0;
    return PM_OK;
}

int pressure_batch_step(pm_batch *b, int32_t *done, void *stream)
{
    if (!b || !done || b->step_pending) return PM_EINVAL;
    // the batch runs on its own stream, after the caller's work so far
    HIPCK(hipEventRecord(b->ev, (hipStream_t)stream));
    HIPCK(hipStreamWaitEvent(b->stream, b->ev, 0));
    TRY(batch_step_impl(b, b->stream));
    for (size_t m = 0; m < b->hs.size(); ++m) done[m] = batch_mesh_done(b, int(m)) ? 1 : 0;
    return PM_OK;
}

int pressure_batch_finish(pm_batch *b, int32_t m, const double *rhs_dev, double rtol, double *p_dev, int32_t *iters,
                          double *true_relres, void *stream)
{
    if (!b || b->step_pending || m < 0 || m >= int(b->hs.size()) || !rhs_dev || !p_dev || !iters || !true_relres) return PM_EINVAL;
    hipStream_t us = (hipStream_t)stream, s = b->stream;
    const int code = batch_finish_impl(b, m, rhs_dev, rtol, p_dev, iters, true_relres, s);
    HIPCK(hipEventRecord(b->ev, s));
    HIPCK(hipStreamWaitEvent(us, b->ev, 0));
    return code;
}

int pressure_batch_solve(pm_batch *b, const double *const *rhs_dev, const double *const *x0_dev, double rtol,
                         int32_t max_iter, double *const *p_dev, int32_t *iters, double *true_relres,
                         int32_t *status, void *stream)
{
    if (!b || b->step_pending || !rhs_dev || !p_dev || !iters || !true_relres || !status || !(rtol > 0.0) ||
        !std::isfinite(rtol) || max_iter < 0)
        return PM_EINVAL;
    const int n = int(b->hs.size());
    for (int m = 0; m < n; ++m)
        if (!rhs_dev[m] || !p_dev[m]) return PM_EINVAL;
    hipStream_t us = (hipStream_t)stream, s = b->stream;
    HIPCK(hipEventRecord(b->ev, us));
    HIPCK(hipStreamWaitEvent(s, b->ev, 0));
    for (int m = 0; m < n; ++m) TRY(batch_begin_impl(b, m, rhs_dev[m], x0_dev ? x0_dev[m] : nullptr, rtol, max_iter, s));
    TRY(batch_refresh(b));
    // every solve stops by itself at max_iter (mixed: within MAX_CORRECTIONS
    // corrections), so this loop is bounded
    const int chunk = std::max(b->graph_iters, 8);
    const int64_t k_limit = int64_t(b->k_next) + int64_t(max_iter) + int64_t(chunk) * (b->mixed ? MAX_CORRECTIONS + 2 : 2) + 2;
    for (;;) {
        TRY(batch_step_impl(b, s));
        int n_done = 0;
        for (int m = 0; m < n; ++m) n_done += batch_mesh_done(b, m) ? 1 : 0;
        if (n_done >= n) break;
        if (b->k_next > k_limit) return PM_EHIP;
    }
    int worst = PM_OK;
    for (int m = 0; m < n; ++m) {
        const int code = batch_finish_impl(b, m, rhs_dev[m], rtol, p_dev[m], &iters[m], &true_relres[m], s);
        status[m] = code;
        if (code < 0 && worst >= 0) worst = code;
        else if (code == PM_NOT_CONVERGED && worst == PM_OK) worst = code;
    }
    HIPCK(hipEventRecord(b->ev, s));
    HIPCK(hipStreamWaitEvent(us, b->ev, 0));
    HIPCK(hipStreamSynchronize(us));
    return worst;
}

int pressure_batch_next_index(pm_batch *b, int32_t *k)
{
    if (!b || !k) return PM_EINVAL;
    *k = b->k_next;
    return PM_OK;
}

}  // extern "C"

// ------------------------------------------------------- projection stage

namespace {

// Dual cells of the handle's mesh, numbered by the sorted tuples of their
// internal (Morton) vertex ids, so that dual-cell arrays follow the order
// in which the kernels visit elements; the caller-facing lists give node
// and element ids in the caller's numbering.
int ensure_faces(pm_handle *h)
{
    if (h->pj.built) return PM_OK;
    const int nv = h->dim + 1, dim = h->dim;
    const int64_t N = h->N, E = h->E;
    std::vector<int4> conn(E);
    std::vector<int32_t> n2o(N);
    HIPCK(hipMemcpy(conn.data(), h->conn, sizeof(int4) * E, hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(n2o.data(), h->new2old, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
    std::vector<int32_t> el(E * nv);
    for (int64_t r = 0; r < E; ++r) {
        const int32_t cv[4] = {conn[r].x, conn[r].y, conn[r].z, conn[r].w};
        for (int a = 0; a < nv; ++a) el[r * nv + a] = cv[a] & 0x7fffffff;
    }
    pm_mesh m{};
    m.dim = h->dim;
    m.n_nodes = N;
    m.n_elems = E;
    m.elems = el.data();
    pm::Faces &F = h->pj.F;
    TRY(pm::build_faces(&m, &F));   // internal vertex and element ids
    const int64_t nf = F.n_faces;
    std::vector<int32_t> efc(E * 4, -1);
    std::vector<uint8_t> ebnd(E, 0);
    for (int64_t r = 0; r < E; ++r)
        for (int a = 0; a < nv; ++a) {
            const int32_t f = F.elem_face[r * nv + a];
            efc[r * 4 + a] = f;
            if (F.elems[2 * int64_t(f) + 1] < 0) ebnd[r] |= uint8_t(1u << a);
        }
    std::vector<int2> fel(nf), fsl(nf);
    h->pj.fv_caller.assign(nf * dim, 0);
    h->pj.fe_caller.assign(nf * 2, -1);
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t x = F.elems[2 * f], y = F.elems[2 * f + 1];
        fel[f] = make_int2(x, y);
        auto slot = [&](int32_t r) {
            for (int a = 0; a < nv; ++a)
                if (efc[int64_t(r) * 4 + a] == f) return int32_t(4 * r + a);
            return int32_t(-1);
        };
        fsl[f] = make_int2(slot(x), y < 0 ? -1 : slot(y));
        int32_t *vc = h->pj.fv_caller.data() + f * dim;
        for (int c = 0; c < dim; ++c) vc[c] = n2o[F.vertices[f * dim + c]];
        std::sort(vc, vc + dim);
        int32_t ex = h->elem_new2old[x], ey = y < 0 ? -1 : h->elem_new2old[y];
        if (ey >= 0 && ey < ex) std::swap(ex, ey);
        h->pj.fe_caller[2 * f] = ex;
        h->pj.fe_caller[2 * f + 1] = ey;
    }
    TRY(dupload(h, &h->pj.efc, efc));
    TRY(dupload(h, &h->pj.fel, fel));
    TRY(dupload(h, &h->pj.fsl, fsl));
    TRY(dupload(h, &h->pj.enew2old, h->elem_new2old));
    TRY(dupload(h, &h->pj.ebnd, ebnd));
    TRY(dalloc(h, &h->pj.e, size_t(10 * E)));
    TRY(dalloc(h, &h->pj.contrib, size_t(4 * E)));
    for (double **v : {&h->pj.pn, &h->pj.gd, &h->pj.b, &h->pj.dp, &h->pj.dpi}) TRY(dalloc(h, v, size_t(N)));
    // the host face lists in internal ids are not needed any more
    std::vector<int32_t>().swap(F.vertices);
    std::vector<int32_t>().swap(F.elems);
    std::vector<int32_t>().swap(F.elem_face);
    h->pj.built = true;
    return PM_OK;
}

template <int DIM, bool PER>
int projection_t(pm_handle *h, const ProjArgs &pa, const double *p_dev, const double *pb_dev, const double *dp0,
                 int32_t n_picard, double rtol, int32_t max_iter, double *p_out, double *wu_out, double *h_out,
                 int32_t *iters, hipStream_t s)
{
    const int N = int(h->N), E = int(h->E), F = int(h->pj.F.n_faces);
    Mesh g = make_mesh<double>(h);
    hipLaunchKernelGGL(k_gather, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, p_dev, h->pj.pn);
    hipLaunchKernelGGL(k_proj_lift, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->dir, pb_dev, h->pj.pn,
                       h->pj.gd);
    // the element passes also write the element part of the next right-hand side
    hipLaunchKernelGGL((k_proj_init<DIM, PER>), dim3(grid_of(E)), dim3(BLK), 0, s, g, pa, h->pj.pn, h->coef,
                       h->pj.gd, h->pj.contrib);
    HIPCK(hipGetLastError());
    TRY(refresh_factors_after_w(h, s));
    int worst = PM_OK;
    const double *x0 = dp0;
    for (int it = 0; it < n_picard; ++it) {
        hipLaunchKernelGGL(k_proj_rhs_node, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->n2e_off, h->n2e_ent, h->dir,
                           h->pj.gd, h->pj.contrib, h->new2old, h->pj.b);
        HIPCK(hipGetLastError());
        int32_t k = 0;
        const int st = pressure_solve(h, h->pj.b, x0, rtol, max_iter, h->pj.dp, &k, nullptr, nullptr, s);
        if (iters) iters[it] = k;
        if (st < 0) return st;
        if (st == PM_NOT_CONVERGED) worst = st;
        x0 = h->pj.dp;
        hipLaunchKernelGGL(k_gather, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, h->pj.dp, h->pj.dpi);
        if (it + 1 < n_picard)
            hipLaunchKernelGGL((k_proj_picard<DIM, PER, true>), dim3(grid_of(E)), dim3(BLK), 0, s, g, pa, h->pj.pn,
                               h->pj.dpi, h->coef, h->pj.gd, h->pj.contrib);
        else
            hipLaunchKernelGGL((k_proj_picard<DIM, PER, false>), dim3(grid_of(E)), dim3(BLK), 0, s, g, pa, h->pj.pn,
                               h->pj.dpi, h->coef, h->pj.gd, h->pj.contrib);
        HIPCK(hipGetLastError());
        TRY(refresh_factors_after_w(h, s));
    }
    hipLaunchKernelGGL(k_proj_faces<DIM>, dim3(grid_of(F)), dim3(BLK), 0, s, F, pa, wu_out);
    hipLaunchKernelGGL(k_add, dim3(grid_of(N)), dim3(BLK), 0, s, N, p_dev, h->pj.dp, p_out);
    if (h_out)
        hipLaunchKernelGGL(k_scatter_elem, dim3(grid_of(E)), dim3(BLK), 0, s, E, h->pj.enew2old, h->coef, h_out);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return worst;
}

}  // namespace

extern "C" {

int pressure_dual_count(pm_handle *h, int64_t *n_faces, int64_t *n_boundary)
{
    if (!h) return PM_EINVAL;
    TRY(ensure_faces(h));
    if (n_faces) *n_faces = h->pj.F.n_faces;
    if (n_boundary) *n_boundary = h->pj.F.n_boundary;
    return PM_OK;
}

int pressure_dual_faces(pm_handle *h, int32_t *face_vertices, int32_t *face_elems)
{
    if (!h) return PM_EINVAL;
    TRY(ensure_faces(h));
    if (face_vertices) std::copy(h->pj.fv_caller.begin(), h->pj.fv_caller.end(), face_vertices);
    if (face_elems) std::copy(h->pj.fe_caller.begin(), h->pj.fe_caller.end(), face_elems);
    return PM_OK;
}

int pressure_projection(pm_handle *h, const double *rho_dev, const double *we_dev, const double *wu_dev,
                        const double *p_dev, const double *pb_dev, const double *bflux_dev,
                        const double *dp0_dev, double gamma, double dt, int32_t n_picard, double rtol,
                        int32_t max_iter, double *p_out, double *wu_out, double *h_out, int32_t *iters,
                        void *stream)
{
    if (!h || !rho_dev || !we_dev || !wu_dev || !p_dev || !p_out || !wu_out) return PM_EINVAL;
    if (!(gamma > 1.0) || !std::isfinite(gamma) || !(dt > 0.0) || !std::isfinite(dt) || n_picard < 1 ||
        !(rtol > 0.0) || !std::isfinite(rtol) || max_iter < 0)
        return PM_EINVAL;
    TRY(ensure_faces(h));
    hipStream_t s = (hipStream_t)stream;
    h->alpha = 1.0 / (gamma - 1.0);
    h->dt = dt;
    TRY(update_v0(h));
    const int64_t E = h->E;
    ProjArgs pa;
    pa.efc = h->pj.efc;
    pa.fel = h->pj.fel;
    pa.ebnd = h->pj.ebnd;
    pa.rho_f = rho_dev;
    pa.we_f = we_dev;
    pa.wu_f = wu_dev;
    pa.bflux = bflux_dev;
    pa.erho = h->pj.e;
    pa.ewe = h->pj.e + E;
    pa.erk = h->pj.e + 2 * E;
    pa.evol = h->pj.e + 3 * E;
    pa.ewu = h->pj.e + 4 * E;
    pa.egrad = h->pj.e + 7 * E;
    pa.g1 = gamma / (gamma - 1.0);
    pa.dt = dt;
    pa.w = h->w;
    auto run = [&]<int DIM, bool PER>() {
        return projection_t<DIM, PER>(h, pa, p_dev, pb_dev, dp0_dev, n_picard, rtol, max_iter, p_out, wu_out, h_out,
                                      iters, s);
    };
    if (h->dim == 2) return h->periodic ? run.template operator()<2, true>() : run.template operator()<2, false>();
    return h->periodic ? run.template operator()<3, true>() : run.template operator()<3, false>();
}

}  // extern "C"

namespace {

int transport_impl(pm_handle *h, const double *rho_dev, const double *wu_dev, const double *we_dev,
                   const double *p_dev, const double *gravity, double c_alpha, double mu, double lambda,
                   double r_gas, double dt, double *rho_out, double *wu_out, double *we_out, bool lader,
                   void *stream)
{
    if (!h || !rho_dev || !wu_dev || !we_dev || !p_dev || !rho_out || !wu_out || !we_out) return PM_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || !(c_alpha >= 0.0) || !std::isfinite(c_alpha)) return PM_EINVAL;
    if (!(mu >= 0.0) || !std::isfinite(mu) || !(lambda >= 0.0) || !std::isfinite(lambda)) return PM_EINVAL;
    if (lambda > 0.0 && (!(r_gas > 0.0) || !std::isfinite(r_gas))) return PM_EINVAL;
    if (rho_out == rho_dev || wu_out == wu_dev || we_out == we_dev) return PM_EINVAL;
    TRY(ensure_faces(h));
    hipStream_t s = (hipStream_t)stream;
    const int N = int(h->N), F = int(h->pj.F.n_faces);
    if (!lader && !h->pj.trec) {
        TRY(dalloc(h, &h->pj.trec, size_t(4) * size_t(F)));
        hipLaunchKernelGGL(k_tr_records, dim3(grid_of(2 * int64_t(F))), dim3(BLK), 0, s, F, h->pj.fsl, h->conn,
                           h->pj.efc, h->pj.trec);
        HIPCK(hipGetLastError());
    }
    const int NG = h->dim + h->dim * h->dim;
    if (lader && !h->pj.grad) TRY(dalloc(h, &h->pj.grad, size_t(NG) * size_t(h->E)));
    if (lader && !h->pj.slots) TRY(dalloc(h, &h->pj.slots, size_t(24) * size_t(h->E)));
    if (lader && !h->pj.oslot) {
        TRY(dalloc(h, &h->pj.oslot, size_t(4) * size_t(h->E)));
        hipLaunchKernelGGL(k_tr_oslot, dim3(grid_of(4 * h->E)), dim3(BLK), 0, s, int(4 * h->E), h->dim + 1, h->pj.efc,
                           h->pj.fsl, h->pj.oslot);
        HIPCK(hipGetLastError());
    }
    TransArgs ta;
    ta.trec = h->pj.trec;
    ta.fsl = h->pj.fsl;
    ta.grad = h->pj.grad;
    ta.oslot = h->pj.oslot;
    ta.rho = rho_dev;
    ta.wu = wu_dev;
    ta.we = we_dev;
    ta.calpha = c_alpha;
    ta.mu = mu;
    ta.lam_r = (lambda > 0.0) ? lambda / r_gas : 0.0;
    ta.dt = dt;
    for (int c = 0; c < 3; ++c) ta.g[c] = (gravity && c < h->dim) ? gravity[c] : 0.0;
    for (int c = 0; c < h->dim; ++c)
        if (!std::isfinite(ta.g[c])) return PM_EINVAL;
    Mesh g = make_mesh<double>(h);
    hipLaunchKernelGGL(k_gather, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, p_dev, h->pj.pn);
    const dim3 grid(grid_of(2 * int64_t(F)));
    auto launch = [&]<int DIM, bool PER>() {
        const bool visc = mu > 0.0 || lambda > 0.0;
        if (lader) {
            hipLaunchKernelGGL((k_tr_grad<DIM, PER>), dim3(grid_of(h->E)), dim3(BLK), 0, s, g, h->pj.efc, rho_dev,
                               wu_dev, h->pj.grad);
            const dim3 eg(grid_of(4 * h->E));
            if (visc)
                hipLaunchKernelGGL((k_lader_elem<DIM, PER, true>), eg, dim3(BLK), 0, s, g, ta, h->pj.efc, h->pj.pn,
                                   h->pj.slots);
            else
                hipLaunchKernelGGL((k_lader_elem<DIM, PER, false>), eg, dim3(BLK), 0, s, g, ta, h->pj.efc, h->pj.pn,
                                   h->pj.slots);
            hipLaunchKernelGGL((k_lader_cell<DIM>), dim3(grid_of(F)), dim3(BLK), 0, s, ta, F, h->pj.slots, rho_out,
                               wu_out, we_out);
        } else if (visc) {
            hipLaunchKernelGGL((k_tr_cell<DIM, PER, true>), grid, dim3(BLK), 0, s, g, ta, h->pj.pn, F, rho_out,
                               wu_out, we_out);
        } else {
            hipLaunchKernelGGL((k_tr_cell<DIM, PER, false>), grid, dim3(BLK), 0, s, g, ta, h->pj.pn, F, rho_out,
                               wu_out, we_out);
        }
    };
    if (h->dim == 2)
        h->periodic ? launch.template operator()<2, true>() : launch.template operator()<2, false>();
    else
        h->periodic ? launch.template operator()<3, true>() : launch.template operator()<3, false>();
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return PM_OK;
}

}  // namespace

extern "C" {

int pressure_transport(pm_handle *h, const double *rho_dev, const double *wu_dev, const double *we_dev,
                       const double *p_dev, const double *gravity, double c_alpha, double mu, double lambda,
                       double r_gas, double dt, double *rho_out, double *wu_out, double *we_out, void *stream)
{
    return transport_impl(h, rho_dev, wu_dev, we_dev, p_dev, gravity, c_alpha, mu, lambda, r_gas, dt, rho_out,
                          wu_out, we_out, false, stream);
}

int pressure_transport_lader(pm_handle *h, const double *rho_dev, const double *wu_dev, const double *we_dev,
                             const double *p_dev, const double *gravity, double c_alpha, double mu, double lambda,
                             double r_gas, double dt, double *rho_out, double *wu_out, double *we_out, void *stream)
{
    return transport_impl(h, rho_dev, wu_dev, we_dev, p_dev, gravity, c_alpha, mu, lambda, r_gas, dt, rho_out,
                          wu_out, we_out, true, stream);
}

}  // extern "C"

extern "C" {

int pressure_post_projection(pm_handle *h, const double *rho_dev, const double *we_dev, const double *wu_dev,
                             const double *p_dev, double gamma, double dt, double *we_out, void *stream)
{
    if (!h || !rho_dev || !we_dev || !wu_dev || !p_dev || !we_out || we_out == we_dev) return PM_EINVAL;
    if (!(gamma > 1.0) || !std::isfinite(gamma) || !(dt > 0.0) || !std::isfinite(dt)) return PM_EINVAL;
    TRY(ensure_faces(h));
    hipStream_t s = (hipStream_t)stream;
    const int N = int(h->N), E = int(h->E), F = int(h->pj.F.n_faces);
    ProjArgs pa{};
    pa.efc = h->pj.efc;
    pa.fel = h->pj.fel;
    pa.ebnd = h->pj.ebnd;
    pa.rho_f = rho_dev;
    pa.we_f = we_dev;
    pa.wu_f = wu_dev;
    pa.evol = h->pj.e + 3 * int64_t(E);
    pa.g1 = gamma / (gamma - 1.0);
    pa.dt = dt;
    double *ewe_new = h->pj.e + 2 * int64_t(E);   // the (rho K) slot, free outside a projection
    Mesh g = make_mesh<double>(h);
    hipLaunchKernelGGL(k_gather, dim3(grid_of(N)), dim3(BLK), 0, s, N, h->new2old, p_dev, h->pj.pn);
    const dim3 ge(grid_of(E));
    if (h->dim == 2 && h->periodic)
        hipLaunchKernelGGL((k_post_elem<2, true>), ge, dim3(BLK), 0, s, g, pa, h->pj.pn, ewe_new);
    else if (h->dim == 2)
        hipLaunchKernelGGL((k_post_elem<2, false>), ge, dim3(BLK), 0, s, g, pa, h->pj.pn, ewe_new);
    else if (h->periodic)
        hipLaunchKernelGGL((k_post_elem<3, true>), ge, dim3(BLK), 0, s, g, pa, h->pj.pn, ewe_new);
    else
        hipLaunchKernelGGL((k_post_elem<3, false>), ge, dim3(BLK), 0, s, g, pa, h->pj.pn, ewe_new);
    hipLaunchKernelGGL(k_post_faces, dim3(grid_of(F)), dim3(BLK), 0, s, F, pa, ewe_new, we_out);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(s));
    return PM_OK;
}

}  // extern "C"

