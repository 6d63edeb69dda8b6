// HIP kernels for gfx950 of the space-time V-cycle.
//
// Streaming kernels (residual, Jacobi update, nodal correction pieces,
// transfers) are HBM-bound: one row of the internal layout holds the N*q
// coefficients of one spatial DOF, so a wavefront (or a 2^k-lane part of it)
// reads a row with consecutive lanes on consecutive 8..128-byte chunks, and
// the DG coupling to slab n-1 stays inside the row (a lane shuffle).
// Reductions use fixed trees, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "factor.hpp"
#include "kernels.hpp"

namespace stmg {

// A launch the library cannot make is an error, not a skipped step.
[[noreturn]] static void fail_launch(const char *what) {
  fprintf(stderr, "stmg: %s\n", what);
  throw StmgError(STMG_EHIP, what);
}

namespace {

constexpr int BLOCK = 256;

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring rows share an L2.
__device__ inline int xcd_remap(int bid, int nblocks) {
  const int x = bid & 7, idx = bid >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  return x * per + min(x, rem) + idx;
}

__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum (256 threads) in a fixed order; result valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double part[BLOCK / 64];
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BLOCK / 64; ++i) s += part[i];
  __syncthreads();
  return s;
}

}  // namespace

// ---------------------------------------------------------------- residual
// r_n = b_n - (K_t (x) M + M_t (x) K) x_n + (N_t (x) M) x_{n-1}
// q = 1: r = b - M(x_n - x_{n-1}) - tau K x_n
// q = 2: with E_{n-1} = (M x)_{n-1,0} + (M x)_{n-1,1} (end value of slab n-1):
//   r0 = b0 - (Mx0 + Mx1) + E_{n-1} - tau K x0
//   r1 = b1 + Mx0 - Mx1 - E_{n-1} - (tau/3) K x1
// Slab-solve right-hand side (mode 1), q = 2: w = (1/2 + i sqrt2/4) r0 - (3 i sqrt2/4) r1
// stored as (re, im) in the two slots of slab n; q = 1: w = r.
// The optional norm (sum of squares of r) is accumulated in FP64.
//
// Lane mapping. A row segment of LPR * C values is read as packets of P = 2
// values (one slab for q = 2): packet p of lane li holds values
// [(p * LPR + li) * P, +P), so every load instruction of a wave covers one
// contiguous run of LPR * P values. The end value of the slab before a
// packet comes from lane li - 1 (same packet) or lane LPR - 1 (packet p - 1).
// Wide rows (N q >= 64 q): one wave per row with the row index wave-uniform,
// so the matrix pattern and values are scalar loads. Rows longer than 64 C
// values (C at most the handle's chunk option) are split into segments, one
// launch per segment in slab order: the set of gathered x rows in flight on
// an XCD is then one segment wide and stays in its L2. Launch s hands the end
// value E of its last slab to launch s + 1 through halo[row] (two alternating
// n_rows arrays). Narrow rows: 64 / LPR rows per wave, one segment.
// Rows are visited in the order sched[] (a space-filling-curve order of the
// edge midpoints): the rows in flight on an XCD then form a compact patch of
// the mesh whose neighbour rows are gathered while still in its L2.
namespace {
template <typename R, int P>
struct Pack;
template <typename R>
struct Pack<R, 1> {
  using type = R;
  __device__ static R get(const type &v, int) { return v; }
  __device__ static void set(type &v, int, R x) { v = x; }
};
template <typename R>
struct Pack<R, 2> {
  using type = R __attribute__((ext_vector_type(2)));
  __device__ static R get(const type &v, int t) { return v[t]; }
  __device__ static void set(type &v, int t, R x) { v[t] = x; }
};
}  // namespace

template <typename R, int C, int Q, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_residual(ResidualArgsT<R> a, int seg, int nseg) {
  constexpr int P = (C % 2 == 0) ? 2 : 1;
  constexpr int NP = C / P;
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int W = a.N * Q;
  const int LPR = WIDE ? 64 : W / C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = WIDE ? lane : lane % LPR;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int gw = blk * (BLOCK / 64) + wave;
  const int slot = WIDE ? gw : gw * (64 / LPR) + lane / LPR;  // position in the visiting order
  const bool active = slot < a.n_rows;
  int row = active && a.sched ? a.sched[slot] : slot;
  if constexpr (WIDE) row = __builtin_amdgcn_readfirstlane(row);
  const int64_t c0 = (int64_t)seg * 64 * C;  // first value of the segment
  R *halo = static_cast<R *>(a.halo);
  const R *hin = seg > 0 ? halo + (int64_t)((seg - 1) & 1) * a.n_rows : nullptr;
  R *hout = seg + 1 < nseg ? halo + (int64_t)(seg & 1) * a.n_rows : nullptr;
  R am[C], ak[C];
#pragma unroll
  for (int j = 0; j < C; ++j) am[j] = ak[j] = 0;
  if (active && a.x) {
    // U nonzeros per step with all their loads issued before the first FMA;
    // the last group repeats the row's last nonzero with weight 0
    constexpr int U = !WIDE ? 4 : (NP >= 8 ? 1 : 8 / NP);
    const int64_t k0 = a.ptr[row], k1 = a.ptr[row + 1];
    for (int64_t k = k0; k < k1; k += U) {
      R mv[U], kv[U];
      V v[U][NP];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = k + u < k1;
        const int64_t kk = in ? k + u : k1 - 1;
        const int c = a.col[kk];
        mv[u] = in ? a.mval[kk] : (R)0;
        kv[u] = in ? a.kval[kk] : (R)0;
        const R *xr = a.x + (int64_t)c * W + c0;
#pragma unroll
        for (int p = 0; p < NP; ++p) v[u][p] = *reinterpret_cast<const V *>(xr + (int64_t)(p * LPR + li) * P);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int t = 0; t < P; ++t) {
            am[p * P + t] += mv[u] * PK::get(v[u][p], t);
            ak[p * P + t] += kv[u] * PK::get(v[u][p], t);
          }
    }
  }
  // end value of the slab before each packet
  const R e_in = (hin && active) ? hin[row] : (R)0;
  R prev[NP];
  R e_last = 0;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    R e = am[p * P + P - 1];
    if constexpr (Q == 2) e += am[p * P];
    const R up = __shfl_up(e, 1, LPR);
    R wrap = e_in;
    if (p > 0) {
      R e1 = am[(p - 1) * P + P - 1];
      if constexpr (Q == 2) e1 += am[(p - 1) * P];
      wrap = __shfl(e1, LPR - 1, LPR);
    }
    prev[p] = li == 0 ? wrap : up;
    e_last = e;
  }
  if (hout && active && lane == 63) hout[row] = e_last;
  double ss = 0.0;
  const R tau = (R)a.tau;
  if (active) {
    const int64_t base = (int64_t)row * W + c0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int64_t off = base + (int64_t)(p * LPR + li) * P;
      const V bv = __builtin_nontemporal_load(reinterpret_cast<const V *>(a.b + off));
      V ov;
      if constexpr (Q == 1) {
        R eprev = prev[p];
#pragma unroll
        for (int t = 0; t < P; ++t) {
          const R r = PK::get(bv, t) - am[p * P + t] + eprev - tau * ak[p * P + t];
          eprev = am[p * P + t];
          PK::set(ov, t, r);
          ss += (double)r * r;
        }
      } else {
        const R m0 = am[2 * p], m1 = am[2 * p + 1];
        const R r0 = PK::get(bv, 0) - (m0 + m1) + prev[p] - tau * ak[2 * p];
        const R r1 = PK::get(bv, 1) + m0 - m1 - prev[p] - (tau / (R)3) * ak[2 * p + 1];
        ss += (double)r0 * r0 + (double)r1 * r1;
        if (a.mode == RES_OUT_SLABRHS) {
          const R s2 = (R)1.4142135623730951;
          PK::set(ov, 0, (R)0.5 * r0);
          PK::set(ov, 1, (R)0.25 * s2 * r0 - (R)0.75 * s2 * r1);
        } else {
          PK::set(ov, 0, r0);
          PK::set(ov, 1, r1);
        }
      }
      __builtin_nontemporal_store(ov, reinterpret_cast<V *>(a.out + off));
    }
  }
  if (a.partial) {
    const double t = block_sum(ss);
    if (threadIdx.x == 0) a.partial[(int64_t)seg * gridDim.x + blockIdx.x] = t;
  }
}

// Grouped residual for wide rows: one wave per group of RES_GROUP rows of
// the visiting order. The wave walks the sorted union of the group's
// neighbour rows and gathers each neighbour's x segment once for every row of
// the group coupled to it (whose mask bit is set; the test is wave-uniform),
// instead of once per nonzero: neighbouring rows along the curve share most
// of their neighbours, so a group of 4 gathers about 40% fewer x
// segments than 4 single rows. Each row sums its nonzeros in ascending
// neighbour order, as the per-row kernel does. Lane mapping, segments, the
// hand-over of end values and the outputs are those of the per-row kernel.
template <typename R, int C, int Q>
__global__ __launch_bounds__(BLOCK) void k_residual_grp(ResidualArgsT<R> a, int seg, int nseg) {
  constexpr int G = RES_GROUP;
  constexpr int P = (C % 2 == 0) ? 2 : 1;
  constexpr int NP = C / P;
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int W = a.N * Q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int grp = __builtin_amdgcn_readfirstlane(blk * (BLOCK / 64) + wave);
  const int ngrp = (a.n_rows + G - 1) / G;
  const bool active = grp < ngrp;
  int row[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int k = grp * G + g;
    row[g] = active && k < a.n_rows ? __builtin_amdgcn_readfirstlane(a.sched[k]) : -1;
  }
  const int64_t c0 = (int64_t)seg * 64 * C;  // first value of the segment
  R *halo = static_cast<R *>(a.halo);
  const R *hin = seg > 0 ? halo + (int64_t)((seg - 1) & 1) * a.n_rows : nullptr;
  R *hout = seg + 1 < nseg ? halo + (int64_t)(seg & 1) * a.n_rows : nullptr;
  // Accumulators. q = 1: am = M x, ak = K x per value. q = 2, per slab
  // (packet) with x0, x1: am[2p] = m0 + m1 (its end value), am[2p+1] = m0 -
  // m1 - (tau/3) k1, ak[p] = -(m0 + m1) - tau k0 (three per slab instead of
  // four: the residual needs no other combination).
  constexpr int CK = Q == 2 ? NP : C;
  const R tau = (R)a.tau, tau3 = tau / (R)3;
  R am[G][C], ak[G][CK];
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int j = 0; j < C; ++j) am[g][j] = 0;
#pragma unroll
    for (int j = 0; j < CK; ++j) ak[g][j] = 0;
  }
  if (active && a.x) {
    // The union entries are read 64 at a time into one register per lane
    // (neighbour row, mask), so the x gathers of a step wait for no other
    // load. U entries per step with all their loads issued before the first
    // FMA; the last step repeats the batch's last entry with an empty mask.
    constexpr int U = NP >= 4 ? 2 : 4;
    const int e0 = a.gptr[grp], e1 = a.gptr[grp + 1];
    for (int eb = e0; eb < e1; eb += 64) {
      const int nbat = min(64, e1 - eb);
      const int my_col = lane < nbat ? a.gent[2 * (eb + lane)] : 0;
      const int my_msk = lane < nbat ? a.gent[2 * (eb + lane) + 1] : 0;
      for (int e = 0; e < nbat; e += U) {
        int msk[U];
        R mv[U][G], kv[U][G];
        V v[U][NP];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool in = e + u < nbat;
          const int j = in ? e + u : nbat - 1;
          const int ee = eb + j;
          const int c = __builtin_amdgcn_readlane(my_col, j);
          msk[u] = in ? __builtin_amdgcn_readlane(my_msk, j) : 0;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            mv[u][g] = a.gval[((int64_t)ee * G + g) * 2];
            kv[u][g] = a.gval[((int64_t)ee * G + g) * 2 + 1];
          }
          const R *xr = a.x + (int64_t)c * W + c0;
#pragma unroll
          for (int p = 0; p < NP; ++p) v[u][p] = *reinterpret_cast<const V *>(xr + (int64_t)(p * 64 + lane) * P);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (!((msk[u] >> g) & 1)) continue;
            if constexpr (Q == 2) {
              const R m = mv[u][g], cp = -m - tau * kv[u][g], cq = -m - tau3 * kv[u][g];
#pragma unroll
              for (int p = 0; p < NP; ++p) {
                const R x0 = PK::get(v[u][p], 0), x1 = PK::get(v[u][p], 1);
                am[g][2 * p] += m * x0;
                am[g][2 * p] += m * x1;
                am[g][2 * p + 1] += m * x0;
                am[g][2 * p + 1] += cq * x1;
                ak[g][p] += cp * x0;
                ak[g][p] -= m * x1;
              }
            } else {
#pragma unroll
              for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int t = 0; t < P; ++t) {
                  am[g][p * P + t] += mv[u][g] * PK::get(v[u][p], t);
                  ak[g][p * P + t] += kv[u][g] * PK::get(v[u][p], t);
                }
            }
          }
      }
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (row[g] < 0) continue;
    // end value of the slab before each packet
    const R e_in = hin ? hin[row[g]] : (R)0;
    R prev[NP];
    R e_last = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const R e = Q == 2 ? am[g][2 * p] : am[g][p * P + P - 1];
      const R up = __shfl_up(e, 1, 64);
      R wrap = e_in;
      if (p > 0) wrap = __shfl(Q == 2 ? am[g][2 * (p - 1)] : am[g][(p - 1) * P + P - 1], 63, 64);
      prev[p] = lane == 0 ? wrap : up;
      e_last = e;
    }
    if (hout && lane == 63) hout[row[g]] = e_last;
    const int64_t base = (int64_t)row[g] * W + c0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int64_t off = base + (int64_t)(p * 64 + lane) * P;
      const V bv = __builtin_nontemporal_load(reinterpret_cast<const V *>(a.b + off));
      V ov;
      if constexpr (Q == 1) {
        R eprev = prev[p];
#pragma unroll
        for (int t = 0; t < P; ++t) {
          const R r = PK::get(bv, t) - am[g][p * P + t] + eprev - tau * ak[g][p * P + t];
          eprev = am[g][p * P + t];
          PK::set(ov, t, r);
          ss += (double)r * r;
        }
      } else {
        const R r0 = PK::get(bv, 0) + ak[g][p] + prev[p];
        const R r1 = PK::get(bv, 1) + am[g][2 * p + 1] - prev[p];
        ss += (double)r0 * r0 + (double)r1 * r1;
        if (a.mode == RES_OUT_SLABRHS) {
          const R s2 = (R)1.4142135623730951;
          PK::set(ov, 0, (R)0.5 * r0);
          PK::set(ov, 1, (R)0.25 * s2 * r0 - (R)0.75 * s2 * r1);
        } else {
          PK::set(ov, 0, r0);
          PK::set(ov, 1, r1);
        }
      }
      __builtin_nontemporal_store(ov, reinterpret_cast<V *>(a.out + off));
    }
  }
  if (a.partial) {
    const double t = block_sum(ss);
    if (threadIdx.x == 0) a.partial[(int64_t)seg * gridDim.x + blockIdx.x] = t;
  }
}

// LDS-tiled residual: one block per tile of RES_TILE rows of the visiting
// order. The tile's matrix entries (neighbour position in the tile's union,
// M and K values) are staged in LDS once; then, segment by segment of
// RES_TILE_SEG values, the union's x rows are staged in LDS with
// coalesced 2-value packets and each row of the tile is computed from there
// (RES_TILE_SEG / 2 lanes per row, every gathered neighbour read from LDS).
// The DG coupling into a segment's first slab uses the row's end value
// carried from the previous segment, so one block does all segments of its
// rows. Each x row is fetched once per tile that needs it (about 3.4 tiles
// per row at RES_TILE = 64) instead of once per nonzero.
template <typename R, int Q>
__global__ __launch_bounds__(BLOCK) void k_residual_tile(ResidualArgsT<R> a) {
  constexpr int NPK = RES_TILE_SEG / 2;  // packets (lanes) per row segment
  constexpr int RPP = BLOCK / NPK;       // rows per pass
  using PK = Pack<R, 2>;
  using V = typename PK::type;
  extern __shared__ __align__(16) unsigned char smem[];
  V *Xs = reinterpret_cast<V *>(smem);                                     // [union][NPK]
  R *Mv = reinterpret_cast<R *>(Xs + (int64_t)a.tile_union_max * NPK);    // [nnz]
  R *Kv = Mv + a.tile_nnz_max;
  R *carry = Kv + a.tile_nnz_max;                                          // [RES_TILE]
  int32_t *rp = reinterpret_cast<int32_t *>(carry + RES_TILE);             // [RES_TILE + 1]
  uint16_t *Lc = reinterpret_cast<uint16_t *>(rp + RES_TILE + 1);          // [nnz]
  const int W = a.N * Q;
  const int nseg = W / RES_TILE_SEG;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int row0 = tile * RES_TILE;
  const int nrow = min(RES_TILE, a.n_rows - row0);
  const int u0 = a.tile_ptr[tile], nu = a.tile_ptr[tile + 1] - u0;
  // stage the tile's matrix entries: row pointers (one wave, prefix sum),
  // then the entries
  if (threadIdx.x < 64) {
    const int k = threadIdx.x;
    int cnt = 0;
    if (k < nrow) {
      const int r = a.sched[row0 + k];
      cnt = (int)(a.ptr[r + 1] - a.ptr[r]);
    }
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (k >= o) incl += t;
    }
    rp[k] = incl - cnt;
    if (k == 63) rp[RES_TILE] = incl;
    carry[k] = (R)0;
  }
  __syncthreads();
  for (int k = threadIdx.x / 4; k < nrow; k += BLOCK / 4) {
    const int r = a.sched[row0 + k];
    const int64_t p0 = a.ptr[r], p1 = a.ptr[r + 1];
    for (int64_t j = p0 + (threadIdx.x & 3); j < p1; j += 4) {
      const int d = rp[k] + (int)(j - p0);
      Lc[d] = a.lcol[j];
      Mv[d] = a.mval[j];
      Kv[d] = a.kval[j];
    }
  }
  const R tau = (R)a.tau;
  double ss = 0.0;
  const int pk = threadIdx.x % NPK, lr = threadIdx.x / NPK;
  for (int seg = 0; seg < nseg; ++seg) {
    __syncthreads();  // previous segment's readers are done with Xs
    const int64_t c0 = (int64_t)seg * RES_TILE_SEG;
    for (int e = threadIdx.x; e < nu * NPK; e += BLOCK) {
      const int u = e / NPK, p = e % NPK;
      Xs[e] = *reinterpret_cast<const V *>(a.x + (int64_t)a.tile_cols[u0 + u] * W + c0 + 2 * p);
    }
    __syncthreads();
    for (int k = lr; k < RES_TILE; k += RPP) {
      const bool active = k < nrow;
      R am0 = 0, am1 = 0, ak0 = 0, ak1 = 0;
      if (active) {
        for (int j = rp[k]; j < rp[k + 1]; ++j) {
          const V v = Xs[(int)Lc[j] * NPK + pk];
          const R mv = Mv[j], kv = Kv[j];
          am0 += mv * PK::get(v, 0);
          am1 += mv * PK::get(v, 1);
          ak0 += kv * PK::get(v, 0);
          ak1 += kv * PK::get(v, 1);
        }
      }
      // end value of this packet's last slab; the previous one from the
      // lane before, or the row's carry for the segment's first packet
      const R e = Q == 2 ? am0 + am1 : am1;
      R prev = __shfl_up(e, 1, NPK);
      if (pk == 0) prev = active ? carry[k] : (R)0;
      if (active && pk == NPK - 1) carry[k] = e;  // read above by this row's lane 0 (same wave)
      if (active) {
        const int r = a.sched[row0 + k];
        const int64_t off = (int64_t)r * W + c0 + 2 * pk;
        const V bv = __builtin_nontemporal_load(reinterpret_cast<const V *>(a.b + off));
        V ov;
        if constexpr (Q == 1) {
          const R r0 = PK::get(bv, 0) - am0 + prev - tau * ak0;
          const R r1 = PK::get(bv, 1) - am1 + am0 - tau * ak1;
          PK::set(ov, 0, r0);
          PK::set(ov, 1, r1);
          ss += (double)r0 * r0 + (double)r1 * r1;
        } else {
          const R r0 = PK::get(bv, 0) - (am0 + am1) + prev - tau * ak0;
          const R r1 = PK::get(bv, 1) + am0 - am1 - prev - (tau / (R)3) * ak1;
          ss += (double)r0 * r0 + (double)r1 * r1;
          if (a.mode == RES_OUT_SLABRHS) {
            const R s2 = (R)1.4142135623730951;
            PK::set(ov, 0, (R)0.5 * r0);
            PK::set(ov, 1, (R)0.25 * s2 * r0 - (R)0.75 * s2 * r1);
          } else {
            PK::set(ov, 0, r0);
            PK::set(ov, 1, r1);
          }
        }
        __builtin_nontemporal_store(ov, reinterpret_cast<V *>(a.out + off));
      }
    }
  }
  if (a.partial) {
    const double t = block_sum(ss);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = t;
  }
}

int64_t residual_tile_lds(int32_t union_max, int32_t nnz_max, int32_t scalar_bytes) {
  const int64_t npk = RES_TILE_SEG / 2;
  return (int64_t)union_max * npk * 2 * scalar_bytes + 2LL * nnz_max * scalar_bytes + RES_TILE * scalar_bytes +
         4LL * (RES_TILE + 1) + 2LL * nnz_max + 16;
}

namespace {
// Values per lane C and rows-per-wave layout of a row of W = N q values.
struct ResShape {
  int C;
  bool wide;
  int nseg;
};
ResShape residual_shape(int W, int q, int chunk) {
  if (W >= 64 * q) {
    const int cmax = std::max(q, chunk > 0 && chunk <= 16 ? chunk : RES_CHUNK_DEFAULT);
    const int C = std::min(W / 64, cmax);
    return {C, true, W / (64 * C)};
  }
  return {q, false, 1};
}
}  // namespace

// Blocks of one segment's launch.
int residual_blocks_per_launch(int32_t n_rows, int32_t W, const ResShape &sh) {
  if (sh.wide) return (n_rows + BLOCK / 64 - 1) / (BLOCK / 64);
  const int rows_per_block = (64 / (W / sh.C)) * (BLOCK / 64);
  return (n_rows + rows_per_block - 1) / rows_per_block;
}

int residual_blocks(int32_t n_rows, int32_t W, int32_t q, int32_t chunk) {
  const ResShape sh = residual_shape(W, q, chunk);
  return residual_blocks_per_launch(n_rows, W, sh) * sh.nseg;
}

template <typename R>
static void launch_residual_inner(const ResidualArgsT<R> &a, int nb, const ResShape &sh, hipStream_t s) {
#define RES_CASE(CC, QQ, WW)                                                                \
  if (sh.C == CC && a.q == QQ && sh.wide == WW) {                                           \
    for (int seg = 0; seg < sh.nseg; ++seg)                                                 \
      hipLaunchKernelGGL((k_residual<R, CC, QQ, WW>), dim3(nb), dim3(BLOCK), 0, s, a, seg,  \
                         sh.nseg);                                                          \
    return;                                                                                 \
  }
  RES_CASE(1, 1, false)
  RES_CASE(1, 1, true)
  RES_CASE(2, 1, true)
  RES_CASE(4, 1, true)
  RES_CASE(8, 1, true)
  RES_CASE(16, 1, true)
  RES_CASE(2, 2, false)
  RES_CASE(2, 2, true)
  RES_CASE(4, 2, true)
  RES_CASE(8, 2, true)
  RES_CASE(16, 2, true)
#undef RES_CASE
  fail_launch("residual: unsupported row shape");
}

// The tiled kernel applies to rows of whole segments with a nonzero x when
// the handle asks for it (chunk RES_CHUNK_TILES) and the mesh has tiles; on
// the 32^3 workload it measured about 2x slower than the per-wave kernel (each
// segment's staging waits behind a barrier), so it is not the default.
template <typename R>
static bool use_tiles(const ResidualArgsT<R> &a) {
  const int W = a.N * a.q;
  return a.chunk == RES_CHUNK_TILES && a.tile_ptr && a.x && a.sched && W % RES_TILE_SEG == 0 &&
         residual_tile_lds(a.tile_union_max, a.tile_nnz_max, sizeof(R)) <= 65536;
}

template <typename R>
static void launch_residual_tiles(const ResidualArgsT<R> &a, hipStream_t s) {
  const int nt = (a.n_rows + RES_TILE - 1) / RES_TILE;
  const size_t lds = (size_t)residual_tile_lds(a.tile_union_max, a.tile_nnz_max, sizeof(R));
  if (a.q == 2)
    hipLaunchKernelGGL((k_residual_tile<R, 2>), dim3(nt), dim3(BLOCK), lds, s, a);
  else
    hipLaunchKernelGGL((k_residual_tile<R, 1>), dim3(nt), dim3(BLOCK), lds, s, a);
}

// Grouped kernel: wide rows with a nonzero x, when the handle provides row
// groups; at most 8 values per lane (the group's accumulators stay in
// registers), longer rows take more segments.
template <typename R>
static bool use_groups(const ResidualArgsT<R> &a) {
  return a.gptr && a.gval && a.x && a.sched && a.chunk != RES_CHUNK_TILES && a.N * a.q >= 64 * a.q;
}

template <typename R>
static void launch_residual_groups(const ResidualArgsT<R> &a, int nb, const ResShape &sh, hipStream_t s) {
#define RESG_CASE(CC, QQ)                                                                       \
  if (sh.C == CC && a.q == QQ) {                                                                \
    for (int seg = 0; seg < sh.nseg; ++seg)                                                     \
      hipLaunchKernelGGL((k_residual_grp<R, CC, QQ>), dim3(nb), dim3(BLOCK), 0, s, a, seg, sh.nseg); \
    return;                                                                                     \
  }
  RESG_CASE(1, 1)
  RESG_CASE(2, 1)
  RESG_CASE(4, 1)
  RESG_CASE(8, 1)
  RESG_CASE(2, 2)
  RESG_CASE(4, 2)
  RESG_CASE(8, 2)
#undef RESG_CASE
  fail_launch("grouped residual: unsupported row shape");
}

template <typename R>
int launch_residual(const ResidualArgsT<R> &a, hipStream_t s) {
  const int W = a.N * a.q;
  if (use_groups(a)) {
    const ResShape sh = residual_shape(W, a.q, a.chunk > 0 && a.chunk < 8 ? a.chunk : 8);
    const int ngrp = (a.n_rows + RES_GROUP - 1) / RES_GROUP;
    const int nb = (ngrp + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0) return 0;
    if (a.prof) {
      char name[64];
      snprintf(name, sizeof name, "k_residual_grp<%s,%d,%d>", sizeof(R) == 8 ? "double" : "float", sh.C, a.q);
      a.prof->begin(s);
      launch_residual_groups(a, nb, sh, s);
      const double rows = a.n_rows, cols = W, nnz = (double)a.nnz, sz = sizeof(R);
      a.prof->end(s, name, 4.0 * nnz * cols, sz * rows * cols * 3.0 + (4.0 + 2.0 * sz) * nnz + 8.0 * (rows + 1));
    } else {
      launch_residual_groups(a, nb, sh, s);
    }
    return nb * sh.nseg;
  }
  if (use_tiles(a)) {
    const int nt = (a.n_rows + RES_TILE - 1) / RES_TILE;
    if (nt == 0) return 0;
    if (a.prof) {
      char name[64];
      snprintf(name, sizeof name, "k_residual_tile<%s,%d>", sizeof(R) == 8 ? "double" : "float", a.q);
      a.prof->begin(s);
      launch_residual_tiles(a, s);
      const double rows = a.n_rows, cols = W, nnz = (double)a.nnz, sz = sizeof(R);
      a.prof->end(s, name, 4.0 * nnz * cols, sz * rows * cols * 3.0 + (4.0 + 2.0 * sz) * nnz + 8.0 * (rows + 1));
      return nt;
    }
    launch_residual_tiles(a, s);
    return nt;
  }
  const ResShape sh = residual_shape(W, a.q, a.chunk);
  const int nb = residual_blocks_per_launch(a.n_rows, W, sh);
  if (nb == 0) return 0;
  if (a.prof) {
    // algorithmic traffic: x, b read once, out written once, the pattern and
    // both value arrays read once; 4 flops per nonzero and column (two FMAs)
    char name[64];
    snprintf(name, sizeof name, "k_residual<%s,%d,%d>", sizeof(R) == 8 ? "double" : "float", sh.C, a.q);
    a.prof->begin(s);
    launch_residual_inner(a, nb, sh, s);
    const double rows = a.n_rows, cols = W, nnz = (double)a.nnz, sz = sizeof(R);
    a.prof->end(s, name, 4.0 * nnz * cols, sz * rows * cols * (a.x ? 3.0 : 2.0) + (4.0 + 2.0 * sz) * nnz + 8.0 * (rows + 1));
    return nb * sh.nseg;
  }
  launch_residual_inner(a, nb, sh, s);
  return nb * sh.nseg;
}
template int launch_residual<double>(const ResidualArgsT<double> &, hipStream_t);
template int launch_residual<float>(const ResidualArgsT<float> &, hipStream_t);

// --------------------------------------------------------------- reductions
__global__ __launch_bounds__(BLOCK) void k_sum(const double *p, int32_t n, double *out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += BLOCK) s += p[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

void launch_sum(const double *partial, int32_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(BLOCK), 0, s, partial, n, out);
}

__global__ __launch_bounds__(BLOCK) void k_sumsq(const double *v, int64_t n, double *partial) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) s += v[i] * v[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

int launch_sumsq(const double *v, int64_t n, double *partial, hipStream_t s) {
  int nb = (int)std::min<int64_t>(2048, (n + BLOCK - 1) / BLOCK);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(BLOCK), 0, s, v, n, partial);
  return nb;
}

// ---------------------------------------------------------- Jacobi update
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_slab_update(int64_t n, int32_t q, R omega, const R *z, R *x,
                                                       int assign) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;  // (row, slab)
  if (i >= n) return;
  if (q == 2) {
    const R zr = z[2 * i], zi = z[2 * i + 1];
    const R d0 = omega * (R)2 * zr, d1 = omega * (R)2 * (zr - (R)1.4142135623730951 * zi);
    if (assign) {
      x[2 * i] = d0;
      x[2 * i + 1] = d1;
    } else {
      x[2 * i] += d0;
      x[2 * i + 1] += d1;
    }
  } else {
    const R d = omega * z[i];
    x[i] = assign ? d : x[i] + d;
  }
}

template <typename R>
void launch_slab_update(int32_t n_rows, int32_t N, int32_t q, double omega, const R *z, R *x, int assign,
                        hipStream_t s) {
  const int64_t n = (int64_t)n_rows * N;
  if (n == 0) return;
  hipLaunchKernelGGL(k_slab_update<R>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, q,
                     (R)omega, z, x, assign);
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_slab_rhs(int64_t n, int32_t q, const R *r, R *w) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  if (q == 2) {
    const R s2 = (R)1.4142135623730951;
    const R r0 = r[2 * i], r1 = r[2 * i + 1];
    w[2 * i] = (R)0.5 * r0;
    w[2 * i + 1] = (R)0.25 * s2 * r0 - (R)0.75 * s2 * r1;
  } else {
    w[i] = r[i];
  }
}

template <typename R>
void launch_slab_rhs(int32_t n_rows, int32_t N, int32_t q, const R *r, R *w, hipStream_t s) {
  const int64_t n = (int64_t)n_rows * N;
  if (n == 0) return;
  hipLaunchKernelGGL(k_slab_rhs<R>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n, q, r, w);
}

// ------------------------------------------------------- nodal correction
// g[v][c] = sum over edges e at v of sign(e, v) r[e][c]  (G^T, entries +-1).
// One thread per 2-value packet of a vertex row (W is even except for
// N = 1, q = 1, which takes the 1-value path); edge lists are broadcast
// loads shared by the lanes of a row.
template <typename R, int P>
__global__ __launch_bounds__(BLOCK) void k_gradT(int32_t n_v, int32_t W, const int64_t *ptr,
                                                 const int32_t *edge, const int8_t *sign, const R *r, R *g) {
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int32_t WP = W / P;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n_v * WP) return;
  const int32_t v = (int32_t)(i / WP), c = (int32_t)(i % WP) * P;
  R acc[P];
#pragma unroll
  for (int t = 0; t < P; ++t) acc[t] = 0;
  const int64_t k1 = ptr[v + 1];
#pragma unroll 4
  for (int64_t k = ptr[v]; k < k1; ++k) {
    const V x = *reinterpret_cast<const V *>(r + (int64_t)edge[k] * W + c);
    const R sg = sign[k] > 0 ? (R)1 : (R)-1;
#pragma unroll
    for (int t = 0; t < P; ++t) acc[t] += sg * PK::get(x, t);
  }
  V out;
#pragma unroll
  for (int t = 0; t < P; ++t) PK::set(out, t, acc[t]);
  *reinterpret_cast<V *>(g + (int64_t)v * W + c) = out;
}

template <typename R>
void launch_gradT(int32_t n_v, int32_t W, const int64_t *ptr, const int32_t *edge, const int8_t *sign,
                  const R *r, R *g, hipStream_t s) {
  const int P = W % 2 == 0 ? 2 : 1;
  const int64_t n = (int64_t)n_v * (W / P);
  if (n == 0) return;
  const dim3 grid((unsigned)((n + BLOCK - 1) / BLOCK));
  if (P == 2)
    hipLaunchKernelGGL((k_gradT<R, 2>), grid, dim3(BLOCK), 0, s, n_v, W, ptr, edge, sign, r, g);
  else
    hipLaunchKernelGGL((k_gradT<R, 1>), grid, dim3(BLOCK), 0, s, n_v, W, ptr, edge, sign, r, g);
}

// One step of the Jacobi-preconditioned Chebyshev iteration for K y = g on
// all W columns of every row (K symmetric in CSR over the rows' numbering,
// dinv = 1 / diag K); a thread per row and packet of P values, as k_gradT:
//   first step (y null): d = b dinv g, y_out = d;
//   later steps:         d = a d + b dinv (g - K y), y_out = y + d.
template <typename R, int P>
__global__ __launch_bounds__(BLOCK) void k_cheb_step(int32_t n, int32_t W, const int64_t *ptr, const int32_t *col,
                                                     const R *val, const R *dinv, const R *g, const R *y, R *d,
                                                     R *y_out, R a, R b) {
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int32_t WP = W / P;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n * WP) return;
  const int32_t v = (int32_t)(i / WP), c = (int32_t)(i % WP) * P;
  const int64_t off = (int64_t)v * W + c;
  const V gv = *reinterpret_cast<const V *>(g + off);
  const R di = dinv[v];
  V dv, yo;
  if (!y) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const R dd = b * di * PK::get(gv, t);
      PK::set(dv, t, dd);
      PK::set(yo, t, dd);
    }
  } else {
    R acc[P];
#pragma unroll
    for (int t = 0; t < P; ++t) acc[t] = 0;
    const int64_t k1 = ptr[v + 1];
#pragma unroll 4
    for (int64_t k = ptr[v]; k < k1; ++k) {
      const V xv = *reinterpret_cast<const V *>(y + (int64_t)col[k] * W + c);
      const R kv = val[k];
#pragma unroll
      for (int t = 0; t < P; ++t) acc[t] += kv * PK::get(xv, t);
    }
    const V d0 = *reinterpret_cast<const V *>(d + off);
    const V y0 = *reinterpret_cast<const V *>(y + off);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const R dd = a * PK::get(d0, t) + b * di * (PK::get(gv, t) - acc[t]);
      PK::set(dv, t, dd);
      PK::set(yo, t, PK::get(y0, t) + dd);
    }
  }
  *reinterpret_cast<V *>(d + off) = dv;
  *reinterpret_cast<V *>(y_out + off) = yo;
}

template <typename R>
void launch_cheb_step(int32_t n, int32_t W, const int64_t *ptr, const int32_t *col, const R *val, const R *dinv,
                      const R *g, const R *y, R *d, R *y_out, double a, double b, hipStream_t s) {
  const int P = W % 2 == 0 ? 2 : 1;
  const int64_t nt = (int64_t)n * (W / P);
  if (nt == 0) return;
  const dim3 grid((unsigned)((nt + BLOCK - 1) / BLOCK));
  if (P == 2)
    hipLaunchKernelGGL((k_cheb_step<R, 2>), grid, dim3(BLOCK), 0, s, n, W, ptr, col, val, dinv, g, y, d, y_out,
                       (R)a, (R)b);
  else
    hipLaunchKernelGGL((k_cheb_step<R, 1>), grid, dim3(BLOCK), 0, s, n, W, ptr, col, val, dinv, g, y, d, y_out,
                       (R)a, (R)b);
}

// Inverse of the time operator on the gradient subspace (K_t on the diagonal,
// -N_t below), per vertex row, in place:
//   q = 1: y_n = sum_{m <= n} g_m (the running sum of eq. (8));
//   q = 2: e_n = sum_{m <= n} g_{m,0}; y_{n,0} = e_{n-1} + (g0 - g1)/2, y_{n,1} = (g0 + g1)/2.
// Same packet mapping as the residual; a wave walks the packets (and, for
// wide rows, the segments) of its row in slab order, scanning across lanes
// and carrying the running sum.
template <typename R, int C, int Q, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_time_scan(int32_t n_v, int32_t N, R *g) {
  constexpr int P = (C % 2 == 0) ? 2 : 1;
  constexpr int NP = C / P;
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int W = N * Q;
  const int LPR = WIDE ? 64 : W / C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = WIDE ? lane : lane % LPR;
  const int gw = blockIdx.x * (BLOCK / 64) + wave;
  const int row = WIDE ? __builtin_amdgcn_readfirstlane(gw) : gw * (64 / LPR) + lane / LPR;
  const bool active = row < n_v;
  const int nseg = WIDE ? W / (64 * C) : 1;
  R carry = 0;
  for (int seg = 0; seg < nseg; ++seg) {
    const int64_t base = (int64_t)row * W + (int64_t)seg * 64 * C;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int64_t off = base + (int64_t)(p * LPR + li) * P;
      V v;
      if (active) {
        v = *reinterpret_cast<const V *>(g + off);
      } else {
#pragma unroll
        for (int t = 0; t < P; ++t) PK::set(v, t, (R)0);
      }
      R local = 0;
      if constexpr (Q == 2) {
        local = PK::get(v, 0);
      } else {
#pragma unroll
        for (int t = 0; t < P; ++t) local += PK::get(v, t);
      }
      R incl = local;
      for (int o = 1; o < LPR; o <<= 1) {
        const R t = __shfl_up(incl, o, LPR);
        if (li >= o) incl += t;
      }
      R e = carry + (incl - local);
      carry += __shfl(incl, LPR - 1, LPR);
      if constexpr (Q == 2) {
        const R g0 = PK::get(v, 0), g1 = PK::get(v, 1);
        PK::set(v, 0, e + (R)0.5 * (g0 - g1));
        PK::set(v, 1, (R)0.5 * (g0 + g1));
      } else {
#pragma unroll
        for (int t = 0; t < P; ++t) {
          e += PK::get(v, t);
          PK::set(v, t, e);
        }
      }
      if (active) *reinterpret_cast<V *>(g + off) = v;
    }
  }
}

template <typename R>
void launch_time_scan(int32_t n_v, int32_t N, int32_t q, R *g, hipStream_t s) {
  const int W = N * q;
  const ResShape sh = residual_shape(W, q, 16);
  const int rows_per_block = sh.wide ? BLOCK / 64 : (64 / (W / sh.C)) * (BLOCK / 64);
  const int nb = (n_v + rows_per_block - 1) / rows_per_block;
  if (nb == 0) return;
#define SCAN_CASE(CC, QQ, WW)                                                                      \
  if (sh.C == CC && q == QQ && sh.wide == WW) {                                                    \
    hipLaunchKernelGGL((k_time_scan<R, CC, QQ, WW>), dim3(nb), dim3(BLOCK), 0, s, n_v, N, g);      \
    return;                                                                                        \
  }
  SCAN_CASE(1, 1, false)
  SCAN_CASE(1, 1, true)
  SCAN_CASE(2, 1, true)
  SCAN_CASE(4, 1, true)
  SCAN_CASE(8, 1, true)
  SCAN_CASE(16, 1, true)
  SCAN_CASE(2, 2, false)
  SCAN_CASE(2, 2, true)
  SCAN_CASE(4, 2, true)
  SCAN_CASE(8, 2, true)
  SCAN_CASE(16, 2, true)
#undef SCAN_CASE
  fail_launch("time scan: unsupported row shape");
}

// x[e][c] += y[head(e)][c] - y[tail(e)][c]  (G, boundary vertices dropped);
// one thread per 2-value packet as in k_gradT.
template <typename R, int P>
__global__ __launch_bounds__(BLOCK) void k_grad_add(int32_t n_e, int32_t W, const int32_t *head,
                                                    const int32_t *tail, const R *y, R *x) {
  using PK = Pack<R, P>;
  using V = typename PK::type;
  const int32_t WP = W / P;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n_e * WP) return;
  const int32_t e = (int32_t)(i / WP), c = (int32_t)(i % WP) * P;
  const int32_t h = head[e], t = tail[e];
  V d;
#pragma unroll
  for (int u = 0; u < P; ++u) PK::set(d, u, (R)0);
  if (h >= 0) d = *reinterpret_cast<const V *>(y + (int64_t)h * W + c);
  if (t >= 0) {
    const V yt = *reinterpret_cast<const V *>(y + (int64_t)t * W + c);
#pragma unroll
    for (int u = 0; u < P; ++u) PK::set(d, u, PK::get(d, u) - PK::get(yt, u));
  }
  V *xp = reinterpret_cast<V *>(x + (int64_t)e * W + c);
  V xv = *xp;
#pragma unroll
  for (int u = 0; u < P; ++u) PK::set(xv, u, PK::get(xv, u) + PK::get(d, u));
  *xp = xv;
}

template <typename R>
void launch_grad_add(int32_t n_e, int32_t W, const int32_t *head, const int32_t *tail, const R *y, R *x,
                     hipStream_t s) {
  const int P = W % 2 == 0 ? 2 : 1;
  const int64_t n = (int64_t)n_e * (W / P);
  if (n == 0) return;
  const dim3 grid((unsigned)((n + BLOCK - 1) / BLOCK));
  if (P == 2)
    hipLaunchKernelGGL((k_grad_add<R, 2>), grid, dim3(BLOCK), 0, s, n_e, W, head, tail, y, x);
  else
    hipLaunchKernelGGL((k_grad_add<R, 1>), grid, dim3(BLOCK), 0, s, n_e, W, head, tail, y, x);
}

// ---------------------------------------------------------------- transfers
// Time prolongation of one coarse slab (coefficients c0, c1) to its halves:
//   first half (c0 - c1/2, c1/2), second half (c0 + c1/2, c1/2); degree 0: (c, c).
// Restriction is its transpose.
template <typename R>
__device__ inline void time_restrict(int q, const R *rf, R *out) {
  // rf: [2][q] fine values of the two halves
  if (q == 1) {
    out[0] = rf[0] + rf[1];
  } else {
    out[0] = rf[0] + rf[2];
    out[1] = (R)0.5 * (-rf[0] + rf[1] + rf[2] + rf[3]);
  }
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_restrict(int32_t n_c, int32_t Nc, int32_t q, const int64_t *ptr,
                                                    const int32_t *col, const double *val, const R *rf,
                                                    R *rc) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;  // (coarse row, coarse slab)
  if (i >= (int64_t)n_c * Nc) return;
  const int32_t row = (int32_t)(i / Nc), m = (int32_t)(i % Nc);
  const int Wf = 2 * Nc * q;
  R acc[2] = {0, 0};
  if (ptr) {
    for (int64_t k = ptr[row]; k < ptr[row + 1]; ++k) {
      R t[2];
      time_restrict(q, rf + (int64_t)col[k] * Wf + 2 * m * q, t);
      acc[0] += (R)val[k] * t[0];
      if (q == 2) acc[1] += (R)val[k] * t[1];
    }
  } else {
    time_restrict(q, rf + (int64_t)row * Wf + 2 * m * q, acc);
  }
  rc[i * q] = acc[0];
  if (q == 2) rc[i * q + 1] = acc[1];
}

template <typename R>
void launch_restrict(int32_t n_c, int32_t Nc, int32_t q, const int64_t *ptr, const int32_t *col,
                     const double *val, const R *r_f, R *r_c, hipStream_t s) {
  const int64_t n = (int64_t)n_c * Nc;
  if (n == 0) return;
  hipLaunchKernelGGL(k_restrict<R>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n_c, Nc, q,
                     ptr, col, val, r_f, r_c);
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_prolong_add(int32_t n_f, int32_t Nc, int32_t q,
                                                       const int64_t *ptr, const int32_t *col,
                                                       const double *val, const R *ec, R *xf) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;  // (fine row, coarse slab)
  if (i >= (int64_t)n_f * Nc) return;
  const int32_t row = (int32_t)(i / Nc), m = (int32_t)(i % Nc);
  const int Wc = Nc * q;
  R c[2] = {0, 0};
  if (ptr) {
    for (int64_t k = ptr[row]; k < ptr[row + 1]; ++k) {
      const R *e = ec + (int64_t)col[k] * Wc + m * q;
      c[0] += (R)val[k] * e[0];
      if (q == 2) c[1] += (R)val[k] * e[1];
    }
  } else {
    const R *e = ec + (int64_t)row * Wc + m * q;
    c[0] = e[0];
    if (q == 2) c[1] = e[1];
  }
  R *x = xf + (int64_t)row * (2 * Wc) + 2 * m * q;
  if (q == 1) {
    x[0] += c[0];
    x[1] += c[0];
  } else {
    x[0] += c[0] - (R)0.5 * c[1];
    x[1] += (R)0.5 * c[1];
    x[2] += c[0] + (R)0.5 * c[1];
    x[3] += (R)0.5 * c[1];
  }
}

template <typename R>
void launch_prolong_add(int32_t n_f, int32_t Nc, int32_t q, const int64_t *ptr, const int32_t *col,
                        const double *val, const R *e_c, R *x_f, hipStream_t s) {
  const int64_t n = (int64_t)n_f * Nc;
  if (n == 0) return;
  hipLaunchKernelGGL(k_prolong_add<R>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, n_f, Nc,
                     q, ptr, col, val, e_c, x_f);
}

// ------------------------------------------------------------------ layout
__global__ __launch_bounds__(BLOCK) void k_abi_to_internal(int32_t n_rows, int32_t W, int32_t ncols,
                                                           const int32_t *map, const double *in,
                                                           double *out) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n_rows * W) return;
  const int32_t row = (int32_t)(i / W), c = (int32_t)(i % W);
  out[i] = in[(int64_t)c * ncols + map[row]];
}

__global__ __launch_bounds__(BLOCK) void k_internal_to_abi(int32_t n_rows, int32_t W, int32_t ncols,
                                                           const int32_t *map, const double *in,
                                                           double *out) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= (int64_t)n_rows * W) return;
  const int32_t row = (int32_t)(i / W), c = (int32_t)(i % W);
  out[(int64_t)c * ncols + map[row]] = in[i];
}

void launch_abi_to_internal(int32_t n_rows, int32_t N, int32_t q, int32_t ncols, const int32_t *map,
                            const double *in, double *out, hipStream_t s) {
  const int64_t n = (int64_t)n_rows * N * q;
  if (n == 0) return;
  hipLaunchKernelGGL(k_abi_to_internal, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                     n_rows, N * q, ncols, map, in, out);
}

void launch_internal_to_abi(int32_t n_rows, int32_t N, int32_t q, int32_t ncols, const int32_t *map,
                            const double *in, double *out, hipStream_t s) {
  const int64_t n = (int64_t)n_rows * N * q;
  if (n == 0) return;
  hipLaunchKernelGGL(k_internal_to_abi, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                     n_rows, N * q, ncols, map, in, out);
}

// b[row][0][k] += psi_k(0) (M u0)[row], psi_0(0) = 1, psi_1(0) = -1
__global__ __launch_bounds__(BLOCK) void k_fold_initial(int32_t n_rows, int32_t W, int32_t q,
                                                        const int64_t *ptr, const int32_t *col,
                                                        const double *mval, const int32_t *map,
                                                        const double *u0, double *b) {
  const int32_t row = blockIdx.x * BLOCK + threadIdx.x;
  if (row >= n_rows) return;
  double acc = 0.0;
  for (int64_t k = ptr[row]; k < ptr[row + 1]; ++k) acc += mval[k] * u0[map[col[k]]];
  b[(int64_t)row * W] += acc;
  if (q == 2) b[(int64_t)row * W + 1] -= acc;
}

void launch_fold_initial(int32_t n_rows, int32_t N, int32_t q, const int64_t *ptr, const int32_t *col,
                         const double *mval, const int32_t *map, const double *u0_abi, double *b,
                         hipStream_t s) {
  if (n_rows == 0) return;
  hipLaunchKernelGGL(k_fold_initial, dim3((n_rows + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, n_rows, N * q,
                     q, ptr, col, mval, map, u0_abi, b);
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_fill(R *p, int64_t n, R v) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename R>
void launch_fill(R *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_fill<R>, dim3(nb), dim3(BLOCK), 0, s, p, n, (R)v);
}

__global__ __launch_bounds__(BLOCK) void k_axpy(int64_t n, double a, const double *x, double *y) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_axpy, dim3(nb), dim3(BLOCK), 0, s, n, a, x, y);
}

// Precision conversions of the refinement loop: out = (float) in, and
// y += (double) x.
__global__ __launch_bounds__(BLOCK) void k_to_float(int64_t n, const double *in, float *out) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) out[i] = (float)in[i];
}
__global__ __launch_bounds__(BLOCK) void k_to_double(int64_t n, const float *in, double *out) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) out[i] = (double)in[i];
}
__global__ __launch_bounds__(BLOCK) void k_add_float(int64_t n, const float *x, double *y) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) y[i] += (double)x[i];
}

void launch_to_float(int64_t n, const double *in, float *out, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(BLOCK), 0, s, n, in, out);
}
void launch_to_double(int64_t n, const float *in, double *out, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_to_double, dim3(nb), dim3(BLOCK), 0, s, n, in, out);
}
void launch_add_float(int64_t n, const float *x, double *y, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(k_add_float, dim3(nb), dim3(BLOCK), 0, s, n, x, y);
}

#define VEC_INST(R)                                                                                         \
  template void launch_slab_update<R>(int32_t, int32_t, int32_t, double, const R *, R *, int, hipStream_t); \
  template void launch_slab_rhs<R>(int32_t, int32_t, int32_t, const R *, R *, hipStream_t);                \
  template void launch_gradT<R>(int32_t, int32_t, const int64_t *, const int32_t *, const int8_t *,        \
                                const R *, R *, hipStream_t);                                              \
  template void launch_time_scan<R>(int32_t, int32_t, int32_t, R *, hipStream_t);                          \
  template void launch_grad_add<R>(int32_t, int32_t, const int32_t *, const int32_t *, const R *, R *,     \
                                   hipStream_t);                                                          \
  template void launch_restrict<R>(int32_t, int32_t, int32_t, const int64_t *, const int32_t *,            \
                                   const double *, const R *, R *, hipStream_t);                          \
  template void launch_prolong_add<R>(int32_t, int32_t, int32_t, const int64_t *, const int32_t *,         \
                                      const double *, const R *, R *, hipStream_t);                       \
  template void launch_fill<R>(R *, int64_t, double, hipStream_t);                                         \
  template void launch_cheb_step<R>(int32_t, int32_t, const int64_t *, const int32_t *, const R *, const R *,  \
                                    const R *, const R *, R *, R *, double, double, hipStream_t);
VEC_INST(double)
VEC_INST(float)
#undef VEC_INST

// ------------------------------------------------------ triangular solves
// Each supernode s stores P_s = [inv(L_ss); -L_{R,s} inv(L_ss)] (m x w,
// column-major). Per tree height, one batched launch does for every
// supernode of that height
//   forward:  [Z[C_s]; U_s] (+)= P_s X[C_s]          (U_s += : update rows)
//   backward: X[C_s] = P_s^T [Z[C_s]; X[R_s]]
// as a GEMM on MFMA (v_mfma_f64_16x16x4f64 in FP64, v_mfma_f32_16x16x4f32
// in FP32; complex products as three real MFMAs). Work items are (supernode, 64-row tile, column tile), the
// column tile varying fastest so the tiles sharing a block of P_s run
// together and read it through L2 once.
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Scalar traits: real type, MFMA accumulator, and the accumulator's lane
// layout (16x16 block: lane l, register r holds column l % 16 of row
// out_row(l, r); the FP64 and FP32 instructions differ here).
template <typename T>
struct Scalar;
template <>
struct Scalar<double> {
  static constexpr bool cpx = false;
  using R = double;
  using acc_t = v4d;
  static constexpr const char *name = "double";
  __device__ static int out_row(int lane, int r) { return 4 * r + lane / 16; }
};
template <>
struct Scalar<cd> {
  static constexpr bool cpx = true;
  using R = double;
  using acc_t = v4d;
  static constexpr const char *name = "cd";
  __device__ static int out_row(int lane, int r) { return 4 * r + lane / 16; }
};
template <>
struct Scalar<float> {
  static constexpr bool cpx = false;
  using R = float;
  using acc_t = v4f;
  static constexpr const char *name = "float";
  __device__ static int out_row(int lane, int r) { return 4 * (lane / 16) + r; }
};
template <>
struct Scalar<cf> {
  static constexpr bool cpx = true;
  using R = float;
  using acc_t = v4f;
  static constexpr const char *name = "cf";
  __device__ static int out_row(int lane, int r) { return 4 * (lane / 16) + r; }
};

__device__ inline v4d mfma_op(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma_op(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename R>
__device__ inline void split(R v, R &re, R &im) {
  re = v;
  im = 0;
}
__device__ inline void split(cd v, double &re, double &im) {
  re = v.re;
  im = v.im;
}
__device__ inline void split(cf v, float &re, float &im) {
  re = v.re;
  im = v.im;
}
template <typename R>
__device__ inline void make(R re, R, R &out) {
  out = re;
}
__device__ inline void make(double re, double im, cd &out) { out = {re, im}; }
__device__ inline void make(float re, float im, cf &out) { out = {re, im}; }

}  // namespace

// Children's contributions to update row i of supernode s, column col, summed
// in the fixed order of the assembly plan (the extend-add of the update rows,
// done where the row is written).
template <typename T, typename R>
__device__ inline void children_sum(const FactorDev &f, const T *U, int s, int i, int32_t nc, int col, R &ur,
                                    R &ui) {
  const int64_t t = f.uasm[s] + i;
  const int64_t k1 = f.asm_tgt[t + 1].src_begin;
  ur = ui = 0;
  for (int64_t k = f.asm_tgt[t].src_begin; k < k1; ++k) {
    R a, b;
    split(U[f.asm_src[k] * nc + col], a, b);
    ur += a;
    ui += b;
  }
}

// Forward assembly (extend-add) of the rows of the supernodes' own columns:
// each target row receives the children's update rows in a fixed order. One
// wavefront per target row.
template <typename T>
__device__ __forceinline__ void fwd_asm_block(const AsmTarget *tgt, int64_t n_tgt, const int64_t *src, int32_t nc,
                                              T *X, T *U, int bid) {
  using R = typename Scalar<T>::R;
  const int64_t ti = (int64_t)bid * (BLOCK / 64) + (threadIdx.x >> 6);
  if (ti >= n_tgt) return;
  const int lane = threadIdx.x & 63;
  const AsmTarget t = tgt[ti];
  const int64_t s1 = tgt[ti + 1].src_begin;
  for (int c = lane; c < nc; c += 64) {
    R ar = 0, ai = 0;
    for (int64_t k = t.src_begin; k < s1; ++k) {
      R r, i;
      split(U[src[k] * nc + c], r, i);
      ar += r;
      ai += i;
    }
    if (t.dst >= 0) {
      R r, i;
      split(X[t.dst * nc + c], r, i);
      make(r + ar, i + ai, X[t.dst * nc + c]);
    } else {
      make(ar, ai, U[(-1 - t.dst) * nc + c]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fwd_asm(const AsmTarget *tgt, int64_t n_tgt, const int64_t *src,
                                                   int32_t nc, T *X, T *U) {
  fwd_asm_block<T>(tgt, n_tgt, src, nc, X, U, blockIdx.x);
}

// Tiles: BM rows x BN columns of the output, K in chunks of KC = 16.
// LDS holds A as [row][k] and B as [col][k] with a row stride of KC + 1
// scalars, which keeps the stores of both load orders and the MFMA operand
// reads free of bank conflicts. Complex products use three real MFMAs
// (re = ArBr - AiBi, im = (Ar+Ai)(Br+Bi) - ArBr - AiBi); LDS holds the real
// and imaginary planes and the sums are formed in registers. The next chunk
// is fetched into registers while the current one is multiplied.
// DIR 0: forward (A = P). DIR 1: backward (A = P^T, read from P), DIR 2:
// backward reading the stored transpose (same access pattern as forward).
// With nsplit > 1 the K range is cut into nsplit segments of kseg and each
// work item writes its partial tile to ws; k_sn_reduce adds them in order
// and applies the epilogue.
// One tile of the launch: bid is the block's index within its launch (its
// position in a grouped launch less the member's first block, a multiple of
// 8, so the XCD placement below is that of a launch of its own).
template <typename T, int BM, int BN, int DIR>
__device__ __forceinline__ void sn_gemm_tile(const FactorDev &f, const SolveTask *tasks, int32_t nc,
                                             int32_t ctiles, T *X, T *Z, T *U, int32_t nsplit, int32_t kseg,
                                             T *ws, int32_t n_rs, int bid) {
  constexpr bool CPX = Scalar<T>::cpx;
  using R = typename Scalar<T>::R;
  using ACC = typename Scalar<T>::acc_t;
  constexpr int NP = CPX ? 3 : 1;  // products: re re, im im, (re + im)(re + im)
  constexpr int NL = CPX ? 2 : 1;  // LDS planes: re, im (the sum plane is formed in registers)
  constexpr int KC = 16, LD = KC + 1;
  constexpr int WN = BN >= 32 ? 2 : 1, WM = 4 / WN;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile shape");
  constexpr int MI = BM / WM / 16, NI = BN / WN / 16;
  constexpr int AE = BM * KC / BLOCK, BE = (BN * KC + BLOCK - 1) / BLOCK;  // elements per thread
  __shared__ R As[NL][BM * LD];
  __shared__ R Bs[NL][BN * LD];
  // Blocks go round-robin to the 8 XCDs (XCD = blockIdx % 8). Row tiles are
  // dealt over the XCDs in turn while all column tiles of one row tile stay
  // on one XCD, consecutive in its dispatch order, so they read the row
  // tile's block of P through one L2. The grid is padded to whole groups of
  // 8 row tiles; blocks past the last row tile exit.
  const int xcd = bid & 7, idx = bid >> 3;
  const int ct = idx % ctiles, rs = (idx / ctiles) * 8 + xcd;
  if (rs >= n_rs) return;
  const int seg = rs % nsplit, rowtile = rs / nsplit;
  const SolveTask task = tasks[rowtile];
  const int s = task.s, rt = task.rt;
  const int c0 = f.col0[s], w = f.col0[s + 1] - c0, m = f.m[s];
  const T *P = reinterpret_cast<const T *>(DIR == 2 ? f.panel_t : f.panel) + f.panel_off[s];
  const int32_t *Rrows = f.rows + f.rptr[s];
  const int i0 = rt * BM, j0 = ct * BN;
  const int rows = DIR == 0 ? m : w;
  const int kb0 = DIR == 0 ? 0 : i0;
  const int ke0 = DIR == 0 ? (i0 < w ? min(w, i0 + BM) : w) : m;
  const int kbeg = nsplit > 1 ? kb0 + seg * kseg : kb0;
  const int kend = nsplit > 1 ? min(ke0, kbeg + kseg) : ke0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / WN) * (BM / WM), wc = (wave % WN) * (BN / WN);

  R ra[AE][2], rb[BE][2];  // prefetch registers (re, im)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      int i, k;
      if (DIR != 1) {  // column segments of P (or of the stored P^T): rows contiguous
        i = e % BM;
        k = e / BM;
      } else {         // P^T rows are P columns: k contiguous
        k = e % KC;
        i = e / KC;
      }
      const int gi = i0 + i, gk = k0 + k;
      ra[q][0] = ra[q][1] = 0;
      if (gi < rows && gk < kend)
        split(DIR == 0 ? P[gi + (int64_t)gk * m] : (DIR == 1 ? P[gk + (int64_t)gi * m] : P[gi + (int64_t)gk * w]),
              ra[q][0], ra[q][1]);
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      const int j = e % BN, k = e / BN;
      const int gk = k0 + k, gj = j0 + j;
      rb[q][0] = rb[q][1] = 0;
      if (k < KC && gk < kend && gj < nc) {
        const T *row;
        if (DIR == 0)
          row = X + (int64_t)(c0 + gk) * nc;
        else
          row = gk < w ? Z + (int64_t)(c0 + gk) * nc : X + (int64_t)Rrows[gk - w] * nc;
        split(row[gj], rb[q][0], rb[q][1]);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      const int i = DIR != 1 ? e % BM : e / KC, k = DIR != 1 ? e / BM : e % KC;
      As[0][i * LD + k] = ra[q][0];
      if constexpr (CPX) As[1][i * LD + k] = ra[q][1];
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      const int j = e % BN, k = e / BN;
      if (k < KC) {
        Bs[0][j * LD + k] = rb[q][0];
        if constexpr (CPX) Bs[1][j * LD + k] = rb[q][1];
      }
    }
  };

  ACC acc[NP][MI][NI];
#pragma unroll
  for (int c = 0; c < NP; ++c)
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
      for (int b = 0; b < NI; ++b) acc[c][a][b] = ACC{0, 0, 0, 0};

  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    stash();
    __syncthreads();
    if (k0 + KC < kend) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + lane / 16;
      R av[NL][MI], bv[NL][NI];
#pragma unroll
      for (int pl = 0; pl < NL; ++pl) {
#pragma unroll
        for (int a = 0; a < MI; ++a) av[pl][a] = As[pl][(wr + a * 16 + (lane & 15)) * LD + kr];
#pragma unroll
        for (int b = 0; b < NI; ++b) bv[pl][b] = Bs[pl][(wc + b * 16 + (lane & 15)) * LD + kr];
      }
#pragma unroll
      for (int pl = 0; pl < NP; ++pl)
#pragma unroll
        for (int a = 0; a < MI; ++a) {
          const R x = pl < 2 ? av[pl < NL ? pl : 0][a] : av[0][a] + av[NL - 1][a];
#pragma unroll
          for (int b = 0; b < NI; ++b) {
            const R y = pl < 2 ? bv[pl < NL ? pl : 0][b] : bv[0][b] + bv[NL - 1][b];
            acc[pl][a][b] = mfma_op(x, y, acc[pl][a][b]);
          }
        }
    }
    __syncthreads();
  }
  // epilogue: lane holds rows out_row(lane, r) of column lane % 16 of each block
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wr + a * 16 + Scalar<T>::out_row(lane, r);
        const int col = j0 + wc + b * 16 + (lane & 15);
        if (nsplit > 1) {  // partial tile: (rowtile, seg) block of BM rows x nc
          if (col >= nc) continue;
          R pr, pi = 0;
          if constexpr (CPX) {
            const R p1 = acc[0][a][b][r], p2 = acc[CPX ? 1 : 0][a][b][r], p3 = acc[CPX ? 2 : 0][a][b][r];
            pr = p1 - p2;
            pi = p3 - p1 - p2;
          } else {
            pr = acc[0][a][b][r];
          }
          make(pr, pi, ws[((int64_t)rs * BM + (row - i0)) * nc + col]);
          continue;
        }
        if (row >= rows || col >= nc) continue;
        R vr, vi = 0;
        if constexpr (CPX) {
          const R p1 = acc[0][a][b][r], p2 = acc[CPX ? 1 : 0][a][b][r], p3 = acc[CPX ? 2 : 0][a][b][r];
          vr = p1 - p2;
          vi = p3 - p1 - p2;
        } else {
          vr = acc[0][a][b][r];
        }
        if (DIR == 0) {
          if (row < w) {
            make(vr, vi, Z[(int64_t)(c0 + row) * nc + col]);
          } else {
            R ur, ui;
            children_sum(f, U, s, row - w, nc, col, ur, ui);
            make(ur + vr, ui + vi, U[(f.uoff[s] + (row - w)) * nc + col]);
          }
        } else {
          make(vr, vi, X[(int64_t)(c0 + row) * nc + col]);
        }
      }
}

template <typename T, int BM, int BN, int DIR>
__global__ __launch_bounds__(BLOCK, 2) void k_sn_gemm(FactorDev f, const SolveTask *tasks,
                                                   int32_t nc, int32_t ctiles, T *X, T *Z, T *U,
                                                   int32_t nsplit, int32_t kseg, T *ws, int32_t n_rs) {
  sn_gemm_tile<T, BM, BN, DIR>(f, tasks, nc, ctiles, X, Z, U, nsplit, kseg, ws, n_rs, blockIdx.x);
}

// Sum of the split-K partial tiles in segment order, then the same epilogue
// as the unsplit kernel (forward: Z rows and U update rows; backward: X[C_s]
// rows). One block per (row tile, chunk of RC columns).
template <typename T, int BM, int DIR>
__device__ __forceinline__ void sn_reduce_block(const FactorDev &f, const SolveTask *tasks, int32_t nc,
                                                int32_t nsplit, const T *ws, T *X, T *Z, T *U, int bid) {
  using R = typename Scalar<T>::R;
  const int RC = nc < 64 ? nc : 64;  // columns per block
  const int cchunks = (nc + RC - 1) / RC;
  const int rowtile = bid / cchunks, cc = bid % cchunks;
  const SolveTask task = tasks[rowtile];
  const int s = task.s, rt = task.rt;
  const int c0 = f.col0[s], w = f.col0[s + 1] - c0;
  const int rows = DIR == 0 ? f.m[s] : w;
  for (int e = threadIdx.x; e < BM * RC; e += BLOCK) {
    const int rr = e / RC, col = cc * RC + e % RC;
    const int row = rt * BM + rr;
    if (row >= rows || col >= nc) continue;
    R ar = 0, ai = 0;
    for (int g = 0; g < nsplit; ++g) {
      R r, i;
      split(ws[(((int64_t)rowtile * nsplit + g) * BM + rr) * nc + col], r, i);
      ar += r;
      ai += i;
    }
    if (DIR != 0) {
      make(ar, ai, X[(int64_t)(c0 + row) * nc + col]);
    } else if (row < w) {
      make(ar, ai, Z[(int64_t)(c0 + row) * nc + col]);
    } else {
      R ur, ui;
      children_sum(f, U, s, row - w, nc, col, ur, ui);
      make(ur + ar, ui + ai, U[(f.uoff[s] + (row - w)) * nc + col]);
    }
  }
}

template <typename T, int BM, int DIR>
__global__ __launch_bounds__(BLOCK) void k_sn_reduce(FactorDev f, const SolveTask *tasks,
                                                     int32_t nc, int32_t nsplit, const T *ws, T *X, T *Z, T *U) {
  sn_reduce_block<T, BM, DIR>(f, tasks, nc, nsplit, ws, X, Z, U, blockIdx.x);
}

// ------------------------------------------------ launches merged over solves
// Several solves (one per member: its factor, plan and right-hand sides) at
// the same step run as one launch: member i owns the blocks
// [block_end[i-1], block_end[i]) and each block runs the tile code of a
// launch of its own with its index within the member. Every output value is
// computed by the same instructions in the same order as in a separate
// launch, so merged and separate solves agree bitwise.
template <typename T>
struct SnGemmArgs {
  FactorDev f;
  const SolveTask *tasks;
  T *X, *Z, *U, *ws;
  int32_t nc, ctiles, nsplit, kseg, n_rs;
};
template <typename T>
struct SnGemmGroup {
  int32_t n;
  int32_t block_end[SOLVE_GROUP_MAX];
  SnGemmArgs<T> m[SOLVE_GROUP_MAX];
};
template <typename T>
struct AsmArgs {
  const AsmTarget *tgt;
  const int64_t *src;
  T *X, *U;
  int64_t n_tgt;
  int32_t nc;
};
template <typename T>
struct AsmGroup {
  int32_t n;
  int32_t block_end[SOLVE_GROUP_MAX];
  AsmArgs<T> m[SOLVE_GROUP_MAX];
};

// Member of the block (wave-uniform) and the block's index within it.
__device__ inline int group_member(const int32_t *block_end, int32_t n, int &bid) {
  int i = 0;
  while (i + 1 < n && (int)blockIdx.x >= block_end[i]) ++i;
  bid = (int)blockIdx.x - (i == 0 ? 0 : block_end[i - 1]);
  return i;
}

template <typename T, int BM, int BN, int DIR>
__global__ __launch_bounds__(BLOCK, 2) void k_sn_gemm_group(SnGemmGroup<T> g) {
  int bid;
  const int i = group_member(g.block_end, g.n, bid);
  const SnGemmArgs<T> &a = g.m[i];
  sn_gemm_tile<T, BM, BN, DIR>(a.f, a.tasks, a.nc, a.ctiles, a.X, a.Z, a.U, a.nsplit, a.kseg, a.ws, a.n_rs, bid);
}

template <typename T, int BM, int DIR>
__global__ __launch_bounds__(BLOCK) void k_sn_reduce_group(SnGemmGroup<T> g) {
  int bid;
  const int i = group_member(g.block_end, g.n, bid);
  const SnGemmArgs<T> &a = g.m[i];
  sn_reduce_block<T, BM, DIR>(a.f, a.tasks, a.nc, a.nsplit, a.ws, a.X, a.Z, a.U, bid);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fwd_asm_group(AsmGroup<T> g) {
  int bid;
  const int i = group_member(g.block_end, g.n, bid);
  const AsmArgs<T> &a = g.m[i];
  fwd_asm_block<T>(a.tgt, a.n_tgt, a.src, a.nc, a.X, a.U, bid);
}

// Launch configuration of one supernode-GEMM launch (tile shape, K split).
struct SnConfig {
  int bmv = 0, bn = 0, ct = 0, nsplit = 1, kseg = 0, dir_k = 0;
  int64_t tiles = 0;
  int32_t n_rs = 0;
  unsigned grid = 0;
  const SolveTask *tasks = nullptr;
};

// Tile shape per launch: BN from the right-hand-side width; 32-row tiles when
// 64-row tiles would leave the GPU short of work items or pad many rows.
template <typename T, int DIR>
static SnConfig sn_config(const FactorDev &f, const SolvePlan::Launch &L, int32_t policy, int32_t splitk,
                          const void *ws, int64_t ws_bytes, int32_t nc) {
  SnConfig c;
  // 32 x 32 tiles for every launch with more than 16 columns: on the 32^3
  // workload they beat the 64-row and 64-column tiles at every tree height
  // (occupancy 5 against 2 waves per SIMD, 4x the work items, less row
  // padding); 64-row tiles only when forced (policy 64)
  int bn = nc > 16 ? 32 : 16;
  bool bm32 = bn == 32;
  if (policy == 64) {
    bm32 = false;
    bn = nc > 32 ? 64 : bn;
  }
  if (policy == 32 && bn >= 32) bm32 = true;
  const int ct = (nc + bn - 1) / bn;
  const SolveTask *tasks = bm32 ? L.tasks32 : L.tasks;
  const int64_t tiles = bm32 ? L.n_tiles32 : L.n_tiles;
  // launches with too few work items for the GPU and long K ranges are split
  // along K (deterministic two-pass sum)
  int nsplit = 1, kseg = 0;
  const int bmv = bm32 ? 32 : 64;
  if (ws && splitk >= 0) {
    int want = 1;
    // forward partial tiles cover all m rows of a front (the update rows
    // too), so the forward splits only launches that leave most of the GPU idle
    // the narrow 64 x 16 tiles (few work items per height) split down to
    // 128-long K ranges until the launch has 4096 work items
    const bool narrow = bn == 16;
    const int64_t fill = narrow ? 4096 : (DIR == 0 ? 512 : 2048);
    if (splitk >= 2)
      want = splitk;
    else if (tiles * ct < fill && L.kmax >= (narrow ? 256 : 512))
      want = (int)std::min<int64_t>(narrow ? 16 : 8, (fill + tiles * ct - 1) / (tiles * ct));
    if (want > 1 && L.kmax > 16) {
      kseg = ((L.kmax + want - 1) / want + 15) / 16 * 16;
      if (narrow && splitk < 2) kseg = std::max(kseg, 128);
      nsplit = (L.kmax + kseg - 1) / kseg;
      if (nsplit < 2 || (int64_t)tiles * nsplit * bmv * nc * (int64_t)sizeof(T) > ws_bytes) nsplit = 1;
    }
  }
  c.n_rs = (int32_t)(tiles * nsplit);  // row tiles x K segments
  c.grid = (unsigned)(((c.n_rs + 7) / 8) * 8 * (int64_t)ct);
  c.dir_k = (DIR == 1 && f.panel_t) ? 2 : DIR;
  c.bmv = bmv;
  c.bn = bn;
  c.ct = ct;
  c.nsplit = nsplit;
  c.kseg = kseg;
  c.tiles = tiles;
  c.tasks = tasks;
  return c;
}

template <typename T, int DIR>
static void launch_sn_gemm(const FactorDev &f, const SolvePlan::Launch &L, int32_t policy, int32_t splitk,
                           Profiler *prof, void *ws, int64_t ws_bytes, int32_t nc, T *X, T *Z, T *U,
                           hipStream_t s) {
  if (L.n_tasks == 0) return;
  const SnConfig c = sn_config<T, DIR>(f, L, policy, splitk, ws, ws_bytes, nc);
  const int bmv = c.bmv, bn = c.bn, ct = c.ct, nsplit = c.nsplit, kseg = c.kseg, dir_k = c.dir_k;
  const int32_t n_rs = c.n_rs;
  const unsigned grid = c.grid;
  const SolveTask *tasks = c.tasks;
  const int64_t tiles = c.tiles;
  // algorithmic work: one multiply-add per structural nonzero of L and
  // right-hand side (8 flops complex, 2 real; the zeros that the dense
  // supernode blocks store are not counted); traffic: those factor entries
  // once, the right-hand-side rows in and out once
  const double scal = (double)sizeof(T);
  // the GEMM launch and the split-K reduce are timed separately; the GEMM
  // carries the launch's algorithmic work (the whole K range), the reduce
  // (named after its GEMM's shape) the partial tiles it reads and the rows
  // it writes
  char name[96], rname[96];
  if (prof) {
    const char *dn = DIR == 0 ? "fwd" : (dir_k == 2 ? "bwdT" : "bwd");
    snprintf(name, sizeof name, "k_sn_gemm<%s,%d,%d,%s>", Scalar<T>::name, bmv, bn, dn);
    snprintf(rname, sizeof rname, "k_sn_reduce<%s,%d,%d,%s>", Scalar<T>::name, bmv, bn, dn);
    prof->begin(s);
  }
  const double flops = (Scalar<T>::cpx ? 8.0 : 2.0) * L.nnz_struct * nc,
               bytes = scal * (L.nnz_struct + 2.0 * L.rows * nc);
  const double rbytes = scal * ((double)nsplit + 1.0) * (double)L.rows * nc;
#define SN_CASE(BMV, BNV)                                                                                  \
  if (bmv == BMV && bn == BNV) {                                                                           \
    if (dir_k == 2)                                                                                        \
      hipLaunchKernelGGL((k_sn_gemm<T, BMV, BNV, 2>), dim3(grid), dim3(BLOCK), 0, s, f, tasks, nc,         \
                         ct, X, Z, U, nsplit, kseg, (T *)ws, n_rs);                                        \
    else                                                                                                   \
      hipLaunchKernelGGL((k_sn_gemm<T, BMV, BNV, DIR>), dim3(grid), dim3(BLOCK), 0, s, f, tasks,             \
                         nc, ct, X, Z, U, nsplit, kseg, (T *)ws, n_rs);                                    \
    if (prof) prof->end(s, name, flops, bytes);                                                            \
    if (nsplit > 1) {                                                                                      \
      if (prof) prof->begin(s);                                                                            \
      hipLaunchKernelGGL((k_sn_reduce<T, BMV, DIR>), dim3((unsigned)(tiles * ((nc + 63) / 64))), dim3(BLOCK), \
                         0, s, f, tasks, nc, nsplit, (const T *)ws, X, Z, U);                               \
      if (prof) prof->end(s, rname, 0.0, rbytes);                                                          \
    }                                                                                                      \
    return;                                                                                                \
  }
  SN_CASE(64, 64)
  SN_CASE(64, 32)
  SN_CASE(64, 16)
  SN_CASE(32, 64)
  SN_CASE(32, 32)
#undef SN_CASE
  if (prof) prof->end(s, name, 0.0, 0.0);
  fail_launch("supernode solve: no kernel for this tile shape");
}

template <typename T>
void solve_forward(const FactorDev &f, const SolvePlan &p, int32_t nc, T *X, T *Z, T *U, hipStream_t s) {
  for (int h = 0; h < p.n_heights; ++h) {
    const int64_t t0 = p.h_tgt_off[h], t1 = p.h_xtgt_end[h];
    if (t1 > t0) {
      if (p.prof) p.prof->begin(s);
      hipLaunchKernelGGL((k_fwd_asm<T>), dim3((unsigned)((t1 - t0 + 3) / 4)), dim3(BLOCK), 0, s, p.tgt + t0,
                         t1 - t0, p.src, nc, X, U);
      if (p.prof) {
        // each source row read once, each target row read and written once
        char name[48];
        snprintf(name, sizeof name, "k_fwd_asm<%s>", Scalar<T>::name);
        const double rows = (double)(p.h_xsrc_end[h] - p.h_src_off[h]) + 2.0 * (double)(t1 - t0);
        p.prof->end(s, name, 0.0, rows * nc * sizeof(T));
      }
    }
    launch_sn_gemm<T, 0>(f, p.fwd[h], p.tile_rows, p.splitk, p.prof, p.splitk_ws, p.splitk_bytes, nc, X, Z, U,
                         s);
  }
}

template <typename T>
void solve_backward(const FactorDev &f, const SolvePlan &p, int32_t nc, T *X, T *Z, hipStream_t s) {
  for (int h = p.n_heights - 1; h >= 0; --h)
    launch_sn_gemm<T, 1>(f, p.bwd[h], p.tile_rows, p.splitk, p.prof, p.splitk_ws, p.splitk_bytes, nc, X, Z,
                         nullptr, s);
}

namespace {
struct GemmItem {
  int member;
  const SolvePlan::Launch *L;
  SnConfig c;
};

// One height of merged solves: GEMM launches grouped by tile shape and
// direction variant, then the split-K reduces of the members that split.
template <typename T, int DIR>
void group_gemm_step(const SolveMember<T> *m, const std::vector<GemmItem> &items, hipStream_t s) {
  std::vector<bool> done(items.size(), false);
  for (size_t a = 0; a < items.size(); ++a) {
    if (done[a]) continue;
    const SnConfig &ca = items[a].c;
    // members of this shape, in chunks of SOLVE_GROUP_MAX
    std::vector<size_t> sel;
    for (size_t b = a; b < items.size(); ++b)
      if (!done[b] && items[b].c.bmv == ca.bmv && items[b].c.bn == ca.bn && items[b].c.dir_k == ca.dir_k) {
        sel.push_back(b);
        done[b] = true;
      }
    for (size_t k0 = 0; k0 < sel.size(); k0 += SOLVE_GROUP_MAX) {
      SnGemmGroup<T> g{};
      SnGemmGroup<T> r{};  // reduces of the members that split along K
      unsigned grid = 0, rgrid = 0;
      for (size_t k = k0; k < std::min(sel.size(), k0 + SOLVE_GROUP_MAX); ++k) {
        const GemmItem &it = items[sel[k]];
        const SolveMember<T> &mm = m[it.member];
        SnGemmArgs<T> arg{*mm.f, it.c.tasks, mm.X, mm.Z, mm.U, (T *)mm.p->splitk_ws, mm.nc, it.c.ct,
                          it.c.nsplit, it.c.kseg, it.c.n_rs};
        grid += it.c.grid;
        g.block_end[g.n] = (int32_t)grid;
        g.m[g.n++] = arg;
        if (it.c.nsplit > 1) {
          rgrid += (unsigned)(it.c.tiles * ((mm.nc + 63) / 64));
          r.block_end[r.n] = (int32_t)rgrid;
          r.m[r.n++] = arg;
        }
      }
      if (grid == 0) continue;
#define SNG_CASE(BMV, BNV)                                                                                   \
  if (ca.bmv == BMV && ca.bn == BNV) {                                                                       \
    if (ca.dir_k == 2)                                                                                       \
      hipLaunchKernelGGL((k_sn_gemm_group<T, BMV, BNV, 2>), dim3(grid), dim3(BLOCK), 0, s, g);               \
    else                                                                                                     \
      hipLaunchKernelGGL((k_sn_gemm_group<T, BMV, BNV, DIR>), dim3(grid), dim3(BLOCK), 0, s, g);             \
    if (r.n > 0) hipLaunchKernelGGL((k_sn_reduce_group<T, BMV, DIR>), dim3(rgrid), dim3(BLOCK), 0, s, r);   \
    continue;                                                                                                \
  }
      SNG_CASE(64, 64)
      SNG_CASE(64, 32)
      SNG_CASE(64, 16)
      SNG_CASE(32, 64)
      SNG_CASE(32, 32)
#undef SNG_CASE
      fail_launch("merged supernode solve: no kernel for this tile shape");
    }
  }
}
}  // namespace

template <typename T>
void solve_forward_group(const SolveMember<T> *m, int n, hipStream_t s) {
  if (n <= 0) return;
  if (n > SOLVE_GROUP_MAX) fail_launch("merged solve: too many members");
  int H = 0;
  for (int i = 0; i < n; ++i) H = std::max(H, m[i].p->n_heights);
  for (int h = 0; h < H; ++h) {
    AsmGroup<T> g{};
    unsigned grid = 0;
    std::vector<GemmItem> items;
    for (int i = 0; i < n; ++i) {
      const SolvePlan &p = *m[i].p;
      if (h >= p.n_heights) continue;
      const int64_t t0 = p.h_tgt_off[h], t1 = p.h_xtgt_end[h];
      if (t1 > t0) {
        grid += (unsigned)((t1 - t0 + 3) / 4);
        g.block_end[g.n] = (int32_t)grid;
        g.m[g.n++] = AsmArgs<T>{p.tgt + t0, p.src, m[i].X, m[i].U, t1 - t0, m[i].nc};
      }
      const SolvePlan::Launch &L = p.fwd[h];
      if (L.n_tasks > 0)
        items.push_back({i, &L, sn_config<T, 0>(*m[i].f, L, p.tile_rows, p.splitk, p.splitk_ws, p.splitk_bytes,
                                                m[i].nc)});
    }
    if (grid > 0) hipLaunchKernelGGL((k_fwd_asm_group<T>), dim3(grid), dim3(BLOCK), 0, s, g);
    group_gemm_step<T, 0>(m, items, s);
  }
}

template <typename T>
void solve_backward_group(const SolveMember<T> *m, int n, hipStream_t s) {
  if (n <= 0) return;
  if (n > SOLVE_GROUP_MAX) fail_launch("merged solve: too many members");
  int H = 0;
  for (int i = 0; i < n; ++i) H = std::max(H, m[i].p->n_heights);
  for (int t = 0; t < H; ++t) {
    std::vector<GemmItem> items;
    for (int i = 0; i < n; ++i) {
      const SolvePlan &p = *m[i].p;
      const int h = p.n_heights - 1 - t;
      if (h < 0) continue;
      const SolvePlan::Launch &L = p.bwd[h];
      if (L.n_tasks > 0)
        items.push_back({i, &L, sn_config<T, 1>(*m[i].f, L, p.tile_rows, p.splitk, p.splitk_ws, p.splitk_bytes,
                                                m[i].nc)});
    }
    group_gemm_step<T, 1>(m, items, s);
  }
}

#define SOLVE_INST(T)                                                                                   \
  template void solve_forward<T>(const FactorDev &, const SolvePlan &, int32_t, T *, T *, T *, hipStream_t); \
  template void solve_backward<T>(const FactorDev &, const SolvePlan &, int32_t, T *, T *, hipStream_t); \
  template void solve_forward_group<T>(const SolveMember<T> *, int, hipStream_t);                       \
  template void solve_backward_group<T>(const SolveMember<T> *, int, hipStream_t);
SOLVE_INST(double)
SOLVE_INST(cd)
SOLVE_INST(float)
SOLVE_INST(cf)
#undef SOLVE_INST

}  // namespace stmg
