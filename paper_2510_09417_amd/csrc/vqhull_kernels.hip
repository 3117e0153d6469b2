// gfx950 kernels of the planar Quickhull (VQhull paper, Algorithm 1).
//
//   k_extremes  leftmost / rightmost point per request (Algorithm 1, first two
//               steps), reading x only; y is read only to break exact x ties.
//   k_sweep     the fused partition pass (Section 3, Section 4 "Bandwidth
//               considerations"): orientation against p->r and r->q, the
//               farthest point of each side, and extraction of S1 / S2, for
//               every tile of every live segment of one recursion level.
//   k_plan0     single-workgroup planner of the roots (p, q of every request).
//   k_finish_plan  one launch per level: workgroup 0 reduces the per-tile
//               results of the level and lays out the next one (breadth-first
//               recursion); every other workgroup finishes whole small
//               subproblems of the level in LDS.
//   k_assemble  clockwise order from the recursion tree (Algorithm 1's
//               unions, in the order p, Hull(S1), q, Hull(S2)).
//   k_small     a single request small enough for the LDS finisher, whole in
//               one launch.
//   k_octagon, k_oct_plan, k_filter, k_filter_scan, k_compact
//               the octagon prefilter (Section 6's Akl-Toussaint heuristic,
//               a variant of the method): eight directional extremes, the
//               points strictly inside their octagon dropped, the rest
//               compacted into the workspace for the top-level passes.
//   k_ingest, k_deinterleave
//               interleaved (x, y) input copied into the workspace.
//   k_gather, k_scatter
//               the batching server's copies in and out of a lane's batch.
//
// Floating point: the orientation value must be bit-identical to the formula
// evaluated operation by operation, so this file is compiled with
// -ffp-contract=off and the pragma below; no fused multiply-add may appear.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "vqhull_internal.h"

#pragma clang fp contract(off)

namespace vqh {

// ------------------------------------------------------------------ helpers

// orient(a, b, c) > 0 iff c is strictly left of a->b (Section 2.1).
__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx, double cy) {
  const double t1 = ax - cx;
  const double t2 = by - cy;
  const double t3 = ay - cy;
  const double t4 = bx - cx;
  const double m1 = t1 * t2;
  const double m2 = t3 * t4;
  return m1 - m2;
}

// Total order of farthest-point candidates: larger key first, then smaller x,
// smaller y, lower index.  kNone loses to every candidate.
//
// Written without branches (bitwise operations on the comparison results): the
// candidate update then lowers to selects.  An equivalent form with early
// returns was lowered wrongly by the gfx950 backend of the ROCm 7.2 compiler
// when the key was a negated orientation value: on lanes that already held a
// candidate the stored key was left unchanged while x, y and the index moved on.
__device__ __forceinline__ bool better(double k, double x, double y, uint32_t i, const Cand& b) {
  const bool tie_y = (y == b.y) & (i < b.i);
  const bool tie_x = (x == b.x) & ((y < b.y) | tie_y);
  const bool ord = (k > b.k) | ((k == b.k) & ((x < b.x) | tie_x));
  return (i != kNone) & ((b.i == kNone) | ord);
}

__device__ __forceinline__ bool better(const Cand& a, const Cand& b) { return better(a.k, a.x, a.y, a.i, b); }

// c = the better of c and o, field by field through selects.
__device__ __forceinline__ void keep(Cand& c, const Cand& o) {
  const bool t = better(o, c);
  c.k = t ? o.k : c.k;
  c.x = t ? o.x : c.x;
  c.y = t ? o.y : c.y;
  c.i = t ? o.i : c.i;
  c.pad = t ? o.pad : c.pad;
}

__device__ __forceinline__ Cand no_cand() {
  Cand c;
  c.k = 0.0;
  c.x = 0.0;
  c.y = 0.0;
  c.i = kNone;
  c.pad = 0;
  return c;
}

__device__ __forceinline__ Cand shfl_xor_cand(const Cand& c, int m) {
  Cand o;
  o.k = __shfl_xor(c.k, m, 64);
  o.x = __shfl_xor(c.x, m, 64);
  o.y = __shfl_xor(c.y, m, 64);
  o.i = __shfl_xor(c.i, m, 64);
  o.pad = __shfl_xor(c.pad, m, 64);
  return o;
}

// Every lane ends with the wave's best candidate.
__device__ __forceinline__ void wave_best(Cand& c) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    keep(c, shfl_xor_cand(c, m));
  }
}

// One DPP step of a wave maximum over doubles: the value from the lane the
// control selects, or the lane's own where there is none (the halves move
// separately).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_fmax(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
  const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
  return fmax(v, __builtin_bit_cast(double, ((uint64_t)ohi << 32) | (uint64_t)olo));
}

__device__ __forceinline__ double readlane_d(double v, int src) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __builtin_bit_cast(double, (hi << 32) | lo);
}

// Largest of a non-negative, non-NaN value over the (fully active) wave, in
// every lane: DPP row shifts 1, 2, 4, 8 and row broadcasts of lanes 15 and
// 31, then lane 63.
__device__ __forceinline__ double wave_max_key(double v) {
  v = dpp_fmax<0x111, 0xf>(v);  // row_shr:1
  v = dpp_fmax<0x112, 0xf>(v);  // row_shr:2
  v = dpp_fmax<0x114, 0xf>(v);  // row_shr:4
  v = dpp_fmax<0x118, 0xf>(v);  // row_shr:8
  v = dpp_fmax<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_fmax<0x143, 0xc>(v);  // row_bcast:31
  return readlane_d(v, 63);
}

// Every lane ends with the wave's best candidate.  Candidates of members have
// keys > 0, so when a single lane holds the wave's largest key its candidate
// is the best and is read from that lane; only exact key ties between lanes
// take the full reduction (among the tied lanes).
__device__ __forceinline__ void wave_best_fast(Cand& c) {
  const bool has = c.i != kNone;
  const double kmax = wave_max_key(has ? c.k : 0.0);
  const bool top = has & (c.k == kmax);
  const unsigned long long m = __ballot(top);
  if (m == 0ull) {
    c = no_cand();
    return;
  }
  if (__popcll(m) == 1) {
    const int src = (int)__builtin_ctzll(m);
    c.k = readlane_d(c.k, src);
    c.x = readlane_d(c.x, src);
    c.y = readlane_d(c.y, src);
    c.i = (uint32_t)__builtin_amdgcn_readlane((int)c.i, src);
    c.pad = (uint32_t)__builtin_amdgcn_readlane((int)c.pad, src);
    return;
  }
  if (!top) c = no_cand();
  wave_best(c);
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// A point (x, y) as one 16-byte value: one load from interleaved input or LDS.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dbl2 d2(double x, double y) {
  dbl2 r;
  r.x = x;
  r.y = y;
  return r;
}

// Values that are the same in every lane (a segment's triangle and range, read
// once per run of tiles) are moved to scalar registers: the loads go through
// the vector memory path, since the compiler cannot prove that the kernel's
// own stores leave them unchanged, and would otherwise hold them in VGPRs.
// (The builtin returns a signed int: each half goes back through uint32_t
// before it is widened.)
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ double uni(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = uni((uint32_t)b);
  const uint64_t hi = uni((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, (hi << 32) | lo);
}

// Lexicographic order of points by (x, y, position); y is loaded only on an
// exact x tie.  ia / ib are positions into y.
__device__ __forceinline__ bool lex_less(double xa, uint32_t ia, double xb, uint32_t ib, const double* y) {
  if (xa != xb) return xa < xb;
  const double ya = y[ia], yb = y[ib];
  if (ya != yb) return ya < yb;
  return ia < ib;
}

// Lexicographic maximum by (x, y), lower position among equal points.
__device__ __forceinline__ bool lex_greater(double xa, uint32_t ia, double xb, uint32_t ib, const double* y) {
  if (xa != xb) return xa > xb;
  const double ya = y[ia], yb = y[ib];
  if (ya != yb) return ya > yb;
  return ia < ib;
}

// ------------------------------------------------------------- k_extremes

// One workgroup per tile of ITER * BLOCK * PPT consecutive points of one
// request (ITER sub-tiles taken in order), one partial record per tile.
template <int BLOCK, int PPT, int ITER>
__global__ __launch_bounds__(BLOCK) void k_extremes(ExtremesArgs A) {
  constexpr uint32_t SUB = BLOCK * PPT;
  constexpr uint32_t TILE = SUB * ITER;
  constexpr int NW = BLOCK / 64;
  __shared__ double s_mnx[NW], s_mxx[NW];
  __shared__ uint32_t s_mni[NW], s_mxi[NW];
  const uint32_t t = blockIdx.x;
  if (t >= A.counts->ext_tiles) return;
  const uint32_t r = A.tile_req ? A.tile_req[t] : 0u;
  const uint32_t off = A.req[r].off, n = A.req[r].n, tile0 = A.req[r].tile0;
  // the request's arrays, indexed by global position (position off = its point 0)
  const double* const X = A.req[r].x - off;
  const double* const Y = A.req[r].y - off;
  const uint32_t lo = off + (t - tile0) * TILE;
  const uint32_t hi = min(off + n, lo + TILE);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  // Branch-free first pass on x alone: a thread's positions increase with
  // (sub-tile, v), so the first strict minimum (maximum) is the lexicographic
  // one unless a later point has exactly the same x; such ties are flagged
  // and that thread's points are taken again with the full order (y, then
  // position).  Positions past the request's end read NaN, which no
  // comparison selects.
  double mnx = __builtin_inf(), mxx = -__builtin_inf();
  uint32_t mni = kNone, mxi = kNone;
  bool bad = false, tmin = false, tmax = false;
  for (int it = 0; it < ITER; ++it) {
    const uint32_t slo = lo + (uint32_t)it * SUB;
    if (slo >= hi) break;  // uniform
    double xs[PPT];
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      xs[v] = pos < hi ? __builtin_nontemporal_load(X + pos) : __builtin_nan("");
    }
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      const double xv = xs[v];
      bad |= (pos < hi) & !finite(xv);
      const bool lt = xv < mnx, gt = xv > mxx;
      tmin = lt ? false : (tmin | (xv == mnx));
      tmax = gt ? false : (tmax | (xv == mxx));
      mnx = lt ? xv : mnx;
      mni = lt ? pos : mni;
      mxx = gt ? xv : mxx;
      mxi = gt ? pos : mxi;
    }
  }
  if (__builtin_expect(__ballot(tmin | tmax) != 0ull, 0)) {
    if (tmin | tmax) {
      mni = mxi = kNone;
      for (uint32_t pos = lo + tid; pos < hi; pos += BLOCK) {
        const double xv = X[pos];
        if (mni == kNone || lex_less(xv, pos, mnx, mni, Y)) {
          mnx = xv;
          mni = pos;
        }
        if (mxi == kNone || lex_greater(xv, pos, mxx, mxi, Y)) {
          mxx = xv;
          mxi = pos;
        }
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double ox = __shfl_xor(mnx, m, 64);
    const uint32_t oi = __shfl_xor(mni, m, 64);
    if (oi != kNone && (mni == kNone || lex_less(ox, oi, mnx, mni, Y))) {
      mnx = ox;
      mni = oi;
    }
    const double gx = __shfl_xor(mxx, m, 64);
    const uint32_t gi = __shfl_xor(mxi, m, 64);
    if (gi != kNone && (mxi == kNone || lex_greater(gx, gi, mxx, mxi, Y))) {
      mxx = gx;
      mxi = gi;
    }
  }
  if (__ballot(bad) && lane == 0) A.req[r].err = 1u;
  if (lane == 0) {
    s_mnx[w] = mnx;
    s_mni[w] = mni;
    s_mxx[w] = mxx;
    s_mxi[w] = mxi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < NW; ++i) {
      if (s_mni[i] != kNone && (mni == kNone || lex_less(s_mnx[i], s_mni[i], mnx, mni, Y))) {
        mnx = s_mnx[i];
        mni = s_mni[i];
      }
      if (s_mxi[i] != kNone && (mxi == kNone || lex_greater(s_mxx[i], s_mxi[i], mxx, mxi, Y))) {
        mxx = s_mxx[i];
        mxi = s_mxi[i];
      }
    }
    ExtPart e;
    e.minx = mnx;
    e.maxx = mxx;
    e.miny = mni != kNone ? Y[mni] : 0.0;
    e.maxy = mxi != kNone ? Y[mxi] : 0.0;
    e.mini = mni != kNone ? mni - off : kNone;
    e.maxi = mxi != kNone ? mxi - off : kNone;
    e.pad[0] = e.pad[1] = 0;
    A.part[t] = e;
  }
}

// ---------------------------------------------------------------- k_sweep
//
// Persistent: gridDim.x workgroups walk the level's tiles (BLOCK*PPT
// consecutive points of one segment each) with stride gridDim.x; the tile
// count comes from the level's status record.  Per tile, each thread loads PPT
// points (striped so that every wave load covers consecutive addresses, with
// non-temporal hints: the data is streamed once), classifies them, and keeps
// the farthest point of each output subset.  Every point's output stream is
// kept as a one-hot byte field; their sums, reduced over the wave, give the
// per-wave subset sizes; one packed 64-bit atomic per output range and tile
// reserves room at the range's left end (first subset) and right end (second
// subset); every wave then writes its survivors as contiguous runs (ranks
// from one wave prefix sum of the one-hot values per point slot, see
// write_onehot).  The order of points inside a subset is irrelevant to the
// result.  Farthest-point candidates are kept per thread across the
// consecutive tiles a workgroup visits in one segment and written once per
// such run.
//
// The orientation values of one point share their coordinate differences:
// orient(a, b, u) = (a.x - u.x) * (b.y - u.y) - (a.y - u.y) * (b.x - u.x), so
// a - u, b - u and r - u are formed once and every predicate is the same two
// rounded products and one rounded difference as the formula evaluated alone.
//
// Modes:
//   kSweepLevel   one recursion level over the workspace (x, y, index), each
//                 segment against its triangle (a, r, b): S1 = left of a->r,
//                 S2 = left of r->b and not in S1 (Algorithm 1's partition).
//   kSweepArgmax  the top level over the caller's arrays, without writing any
//                 point: only the sizes and farthest points of S1 = left of
//                 p->q and S2 = left of q->p (orient(q, p, u) is exactly
//                 -orient(p, q, u)).
//   kSweepFused   the caller's arrays again: each point is classified against
//                 p->q and then against the triangle of the child it falls in,
//                 (p, r1, q) or (q, r2, p), so the top level's subsets are
//                 never written or read back.  Children small enough for the
//                 LDS finisher are copied instead (pass-through).
//   kSweepArgmaxWs, kSweepFusedWs
//                 the same two passes over the points the octagon prefilter
//                 kept (buffer A, indices from its index array).
//   kSweepArgmaxPair, kSweepFusedPair
//                 the same two passes below the top (a level pair, for levels
//                 that keep most of their points): the workspace's segments
//                 (a, r, b) with Algorithm 1's partition, S1 = left of a->r,
//                 S2 = left of r->b and not in S1; the argmax pass writes
//                 nothing, the fused pass re-reads the segment and writes the
//                 subsets of its children (a, r1, r) and (r, r2, b).

// Per-thread farthest-point candidate inside a sweep: the key and the position
// of the point in the level's input arrays.  Coordinates and index are fetched
// only when a run of tiles is flushed, or when two keys are exactly equal.
// Members of a subset have keys > 0, so key 0 with position kNone ("none")
// loses every comparison on the key alone.
struct Best {
  double k;
  uint32_t pos;
};

__device__ __forceinline__ Best no_best() {
  Best b;
  b.k = 0.0;
  b.pos = kNone;
  return b;
}

// The arrays a sweep reads its points from: coordinates, and in the workspace
// the request-local index of every position (the caller's arrays carry none:
// there the index is the position minus the request's first position).
struct Src {
  const double* x;
  const double* y;
  const uint32_t* i;
};

__device__ __forceinline__ const double* uni_ptr(const double* p) {
  const uint64_t b = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = uni((uint32_t)b), hi = uni((uint32_t)(b >> 32));
  return reinterpret_cast<const double*>((hi << 32) | lo);
}

// Ordering of two members with equal keys (the stored one at position b.pos):
// smaller x, then smaller y, then lower index.  In the caller's arrays the
// index order is the position order.
template <bool USER>
__device__ __forceinline__ bool tie_wins(const Src& A, double x, double y, uint32_t pos, uint32_t idx,
                                         uint32_t bpos) {
  const double bx = A.x[bpos], by = A.y[bpos];
  const uint32_t bi = USER ? bpos : A.i[bpos];
  const uint32_t ni = USER ? pos : idx;
  return (x < bx) | ((x == bx) & ((y < by) | ((y == by) & (ni < bi))));
}

// Offer NB points (one per candidate slot q, flag in[q], key k[q]) that share
// the coordinates (x, y) and position pos.  Exact key ties are rare: they take
// a wave-uniform slow path that fetches the stored candidate's coordinates.
template <bool USER, int NB>
__device__ __forceinline__ void offer(Best (&b)[NB], const bool (&in)[NB], const double (&k)[NB], double x, double y,
                                      uint32_t pos, uint32_t idx, const Src& A) {
  bool t[NB], tie[NB];
  bool any_tie = false;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    t[q] = in[q] & (k[q] > b[q].k);
    tie[q] = in[q] & (k[q] == b[q].k);
    any_tie |= tie[q];
  }
  if (__builtin_expect(__ballot(any_tie) != 0ull, 0)) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (tie[q]) t[q] = tie_wins<USER>(A, x, y, pos, idx, b[q].pos);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    b[q].k = t[q] ? k[q] : b[q].k;
    b[q].pos = t[q] ? pos : b[q].pos;
  }
}

template <bool USER>
__device__ __forceinline__ Cand to_cand(const Src& A, const Best& b, uint32_t ibase) {
  Cand c = no_cand();
  if (b.pos != kNone) {
    c.k = b.k;
    c.x = A.x[b.pos];
    c.y = A.y[b.pos];
    c.i = USER ? b.pos - ibase : A.i[b.pos];
  }
  return c;
}

// The wave's best candidate.  Only lanes whose key equals the wave's largest
// key fetch their point (one cache line, not one per lane); several such lanes
// are ordered by the full tie-break.
template <bool USER>
__device__ __forceinline__ Cand wave_cand(const Src& A, const Best& b, uint32_t ibase) {
  const double kmax = wave_max_key(b.k);  // keys are >= 0: no NaN
  Cand c = no_cand();
  if (b.pos != kNone && b.k == kmax) c = to_cand<USER>(A, b, ibase);
  wave_best_fast(c);
  return c;
}

// Best candidates of a run over the workgroup, written to record slot `slot`.
template <bool USER, int NW>
__device__ __forceinline__ void flush_run(const Src& A, TilePart* part, uint32_t slot, const Best& b1,
                                          const Best& b2, uint32_t ibase, Cand (*s_cand)[NW]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Cand c1 = wave_cand<USER>(A, b1, ibase), c2 = wave_cand<USER>(A, b2, ibase);
  if (lane == 0) {
    s_cand[0][w] = c1;
    s_cand[1][w] = c2;
  }
  __syncthreads();
  if (tid == 0) {
    Cand r1 = s_cand[0][0], r2 = s_cand[1][0];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      keep(r1, s_cand[0][i]);
      keep(r2, s_cand[1][i]);
    }
    part[slot].c[0] = r1;
    part[slot].c[1] = r2;
  }
  __syncthreads();
}

// Sum of a value over the (fully active) wave, returned in a scalar register:
// an inclusive prefix sum by DPP row shifts 1, 2, 4, 8 (within rows of 16
// lanes) and row broadcasts of lanes 15 and 31; lane 63 ends with the total.
// Lanes without a valid source add the zero passed as "old".
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;  // lane i: the sum over lanes 0..i
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_incl(v), 63);
}

// Argmax pass: add a run's subset sizes (per lane) to the segment's counter,
// one atomic per workgroup.
template <int NW>
__device__ __forceinline__ void flush_counts(unsigned long long* ctr, uint32_t run1, uint32_t run2,
                                             uint32_t (*s_cnt)[NW]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t t1 = wave_sum(run1), t2 = wave_sum(run2);
  if (lane == 0) {
    s_cnt[0][w] = t1;
    s_cnt[1][w] = t2;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long a = 0ull, b = 0ull;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      a += s_cnt[0][i];
      b += s_cnt[1][i];
    }
    if (a | b) atomicAdd(ctr, (b << 32) | a);
  }
  __syncthreads();
}

// Reserve room for one tile's survivors and write them (one-hot form).
// oh[v] holds, for the thread's v-th point, 1 << (8 s) if it goes to stream s
// (s < NS), else 0.  Stream s goes to the left end (even s) or the right end
// (odd s) of output range s / 2.  Per v, one wave prefix sum of the packed
// one-hot values gives every lane its rank in its own stream; lane s of a
// per-wave table holds stream s's next write position.
template <int BLOCK, int PPT, int NS, bool USER>
__device__ __forceinline__ void write_onehot(const uint32_t (&oh)[PPT], const uint32_t (&beg)[NS / 2],
                                             const uint32_t (&cnt)[NS / 2], unsigned long long* const (&ctr)[NS / 2],
                                             const double (&px)[PPT], const double (&py)[PPT],
                                             const uint32_t (&pi)[PPT], uint32_t idx0, double* ox, double* oy,
                                             uint32_t* oi, uint32_t (*s_cnt)[BLOCK / 64], uint32_t* s_base) {
  constexpr int NW = BLOCK / 64;
  constexpr int NR = NS / 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t c = 0;  // per-lane stream sizes, 8-bit fields (at most PPT each)
#pragma unroll
  for (int v = 0; v < PPT; ++v) c += oh[v];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const uint32_t pair = ((c >> (16 * j)) & 0xFFu) | (((c >> (16 * j + 8)) & 0xFFu) << 16);
    const uint32_t both = wave_sum(pair);
    if (lane == 0) {
      s_cnt[2 * j][w] = both & 0xFFFFu;
      s_cnt[2 * j + 1][w] = both >> 16;
    }
  }
  __syncthreads();
  if (tid < NR) {
    const int j = tid;
    uint32_t t1 = 0, t2 = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t a = s_cnt[2 * j][i], b = s_cnt[2 * j + 1][i];
      s_cnt[2 * j][i] = t1;
      s_cnt[2 * j + 1][i] = t2;
      t1 += a;
      t2 += b;
    }
    unsigned long long* cp = ctr[0];
    uint32_t b0 = beg[0], n0 = cnt[0];
    if (NR > 1 && j == 1) {
      cp = ctr[NR - 1];
      b0 = beg[NR - 1];
      n0 = cnt[NR - 1];
    }
    unsigned long long old = 0ull;
    if (t1 | t2) old = atomicAdd(cp, ((unsigned long long)t2 << 32) | (unsigned long long)t1);
    s_base[2 * j] = b0 + (uint32_t)old;
    s_base[2 * j + 1] = b0 + n0 - (uint32_t)(old >> 32) - t2;
  }
  __syncthreads();
  const int ls = lane < NS ? lane : 0;
  uint32_t tab = lane < NS ? s_base[ls] + s_cnt[ls][w] : 0u;  // lane s < NS: stream s's next position
  const uint32_t lsh = (uint32_t)(8 * (lane & 3));
#pragma unroll
  for (int v = 0; v < PPT; ++v) {
    const uint32_t h = oh[v];
    const uint32_t incl = wave_scan_incl(h);
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t sh = h ? (uint32_t)__builtin_ctz(h) : 0u;  // 8 s
    const uint32_t base = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(sh >> 1), (int)tab);
    if (h) {
      const uint32_t dst = base + ((incl >> sh) & 0xFFu) - 1u;
      ox[dst] = px[v];  // plain stores: the L2 merges the partial lines of
      oy[dst] = py[v];  // neighbouring runs before they reach HBM
      oi[dst] = USER ? idx0 + (uint32_t)(v * BLOCK) : pi[v];
    }
    tab += (tot >> lsh) & 0xFFu;
  }
}

template <int BLOCK, int PPT, int MODE>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs A) {
  static_assert(PPT <= 32, "class masks are 32-bit");
  // USER: input = the caller's arrays, index = position - ibase
  constexpr bool USER = MODE == kSweepArgmax || MODE == kSweepFused;
  constexpr bool FUSED = MODE == kSweepFused || MODE == kSweepFusedWs || MODE == kSweepFusedPair;
  constexpr bool ARGMAX = MODE == kSweepArgmax || MODE == kSweepArgmaxWs || MODE == kSweepArgmaxPair;
  constexpr bool PAIR = MODE == kSweepArgmaxPair || MODE == kSweepFusedPair;  // a segment (a, r, b), not a root
  constexpr int NS = FUSED ? 4 : 2;  // output streams (two per output range)
  constexpr uint32_t TILE = BLOCK * PPT;
  constexpr int NW = BLOCK / 64;
  __shared__ uint32_t s_cnt[NS][NW];
  __shared__ uint32_t s_base[NS];
  __shared__ Cand s_cand[2][NW];

  const uint32_t ntiles = uni(A.st->ntiles);
  const uint32_t G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  uint32_t run_seg = kNone, run_slot = 0;
  Src src{A.ix, A.iy, A.ii};  // USER: replaced per segment by its request's own arrays
  // Level: the segment's triangle (a, r, b).  Argmax and fused: p = a, q = r.
  double ax = 0, ay = 0, rx = 0, ry = 0, bx = 0, by = 0;
  double r1x = 0, r1y = 0, r2x = 0, r2y = 0;  // fused: farthest points of the two children
  double vr1x = 0, vr1y = 0, vr2x = 0, vr2y = 0;  // the same in vector registers (selected per lane)
  uint32_t beg = 0, cnt = 0, tile0 = 0, ibase = 0, req = 0;
  uint32_t cbeg[NS / 2] = {}, ccnt[NS / 2] = {};
  unsigned long long* cctr[NS / 2] = {};
  bool split0 = false, split1 = false, copy0 = false, copy1 = false;  // fused: kinds of the two children
  Best b[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) b[s] = no_best();
  uint32_t run1 = 0, run2 = 0;  // argmax pass: subset sizes of the current run (per lane)
  bool bad = false;

  for (uint32_t k = blockIdx.x; k < ntiles; k += G) {
    const uint32_t t = A.reverse ? ntiles - 1u - k : k;
    const uint32_t s = uni(A.tile_seg[t]);
    if (s != run_seg) {
      if (run_seg != kNone) {
        flush_run<USER, NW>(src, A.part, run_slot, b[0], b[1], ibase, s_cand);
        if constexpr (FUSED) flush_run<USER, NW>(src, A.part2, run_slot, b[2], b[3], ibase, s_cand);
        if constexpr (ARGMAX) {
          flush_counts<NW>(A.ctr + (size_t)run_seg * kCtrStride, run1, run2, s_cnt);
          run1 = run2 = 0;
        }
      }
      if constexpr (FUSED) {
        const FusedRoot* fr = A.fr + s;
        ax = uni(fr->px);
        ay = uni(fr->py);
        rx = uni(fr->qx);
        ry = uni(fr->qy);
        if constexpr (PAIR) {
          bx = uni(fr->bx);
          by = uni(fr->by);
        }
        r1x = uni(fr->rx[0]);
        r1y = uni(fr->ry[0]);
        r2x = uni(fr->rx[1]);
        r2y = uni(fr->ry[1]);
        vr1x = r1x;
        vr1y = r1y;
        vr2x = r2x;
        vr2y = r2y;
        asm volatile("" : "+v"(vr1x), "+v"(vr1y), "+v"(vr2x), "+v"(vr2y));
        beg = uni(fr->off);
        cnt = uni(fr->n);
        tile0 = uni(fr->tile0);
        ibase = beg;
        req = uni(fr->req);
        uint32_t kind[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          cbeg[c] = uni(fr->beg[c]);
          ccnt[c] = uni(fr->cnt[c]);
          kind[c] = uni(fr->kind[c]);
          cctr[c] = (kind[c] == kFuseSplit ? A.ctr : A.jctr) + (size_t)uni(fr->slot[c]) * kCtrStride;
        }
        split0 = kind[0] == kFuseSplit;
        split1 = kind[1] == kFuseSplit;
        copy0 = kind[0] == kFuseCopy;
        copy1 = kind[1] == kFuseCopy;
      } else {
        const Seg* sg = A.seg + s;
        ax = uni(sg->ax);
        ay = uni(sg->ay);
        rx = uni(sg->rx);
        ry = uni(sg->ry);
        bx = uni(sg->bx);
        by = uni(sg->by);
        beg = uni(sg->beg);
        cnt = uni(sg->cnt);
        tile0 = uni(sg->tile0);
        ibase = uni(sg->ibase);
        req = uni(sg->req);
        cbeg[0] = beg;
        ccnt[0] = cnt;
        cctr[0] = A.ctr + (size_t)s * kCtrStride;
      }
      if constexpr (USER) {  // positions are global; the request's point 0 sits at position ibase
        src.x = uni_ptr(A.req[req].x) - ibase;
        src.y = uni_ptr(A.req[req].y) - ibase;
      }
      run_seg = s;
      run_slot = tile0 + (t - tile0) % G;
#pragma unroll
      for (int q = 0; q < NS; ++q) b[q] = no_best();
    }
    const uint32_t lo = beg + (t - tile0) * TILE;
    const uint32_t hi = min(beg + cnt, lo + TILE);

    // Loads: positions past the end of the segment re-read its last point
    // (no branch per load) and are masked out below.
    double px[PPT], py[PPT];
    uint32_t pi[PPT];
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pc = min(lo + v * BLOCK + tid, hi - 1u);
      px[v] = __builtin_nontemporal_load(src.x + pc);
      py[v] = __builtin_nontemporal_load(src.y + pc);
      if constexpr (USER) {
        pi[v] = 0u;
      } else {
        pi[v] = __builtin_nontemporal_load(src.i + pc);
      }
    }

    uint32_t m[2] = {0u, 0u};  // argmax pass: bit v set for the thread's v-th point in S1 / S2
    uint32_t oh[PPT];          // the other passes: each point's output stream, one-hot (write_onehot)
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = lo + v * BLOCK + tid;
      const bool ok = pos < hi;
      const double x = px[v], y = py[v];
      if constexpr (MODE == kSweepLevel) {
        const double dax = ax - x, day = ay - y, drx = rx - x, dry = ry - y, dbx = bx - x, dby = by - y;
        const double o1 = dax * dry - day * drx;  // orient(a, r, u)
        const double o2 = drx * dby - dry * dbx;  // orient(r, b, u)
        const bool in1 = ok & (o1 > 0.0);
        const bool in2 = ok & !in1 & (o2 > 0.0);
        const bool f[2] = {in1, in2};
        const double kk[2] = {o1, o2};
        offer<false, 2>(b, f, kk, x, y, pos, pi[v], src);
        oh[v] = (in1 ? 1u : 0u) | (in2 ? 256u : 0u);
      } else {
        const double dpx = ax - x, dpy = ay - y, dqx = rx - x, dqy = ry - y;
        const double o = dpx * dqy - dpy * dqx;  // orient(p, q, u); a pair: orient(a, r, u)
        // A root's S2 = left of q->p: orient(q, p, u) is exactly -o.  A pair's
        // S2 = left of r->b and not in S1.
        double o2 = -o, dbx = 0.0, dby = 0.0;
        if constexpr (PAIR) {
          dbx = bx - x;
          dby = by - y;
          o2 = dqx * dby - dqy * dbx;  // orient(r, b, u)
        }
        const bool s0 = ok & (o > 0.0);
        const bool s1 = PAIR ? (ok & !(o > 0.0) & (o2 > 0.0)) : (ok & (o < 0.0));
        if constexpr (ARGMAX) {
          const bool f[2] = {s0, s1};
          const double kk[2] = {o, o2};
          offer<USER, 2>(b, f, kk, x, y, pos, pi[v], src);
          m[0] |= (uint32_t)s0 << v;
          m[1] |= (uint32_t)s1 << v;
          if constexpr (USER) bad |= ok & !finite(y);  // the octagon pass checked the kept points
        } else {
          // child 0 = (p, r1, q) holds S1, child 1 = (q, r2, p) holds S2.  Both
          // children are evaluated for every point (no branch on the kinds,
          // which are uniform); the kind flags mask the results.
          // The point's own child only: R = r1 for S1 (child (p, r1, q)),
          // r2 for S2 (child (q, r2, p)).  With d = R - u,
          //   U = orient(p, R, u) = (p.x-u.x)(R.y-u.y) - (p.y-u.y)(R.x-u.x)
          //   V = orient(q, R, u) = (q.x-u.x)(R.y-u.y) - (q.y-u.y)(R.x-u.x);
          // orient(r1, q, u) has the same two rounded products in the other
          // order, so it is exactly -V; likewise orient(r2, p, u) = -U.
          // A pair's child 1 is (r, r2, b): U = orient(b, R, u) there, so that
          // -U = orient(r2, b, u) exactly (a root's b is p).
          const double dRx = (s0 ? vr1x : vr2x) - x, dRy = (s0 ? vr1y : vr2y) - y;
          const double dPx = PAIR ? (s0 ? dpx : dbx) : dpx, dPy = PAIR ? (s0 ? dpy : dby) : dpy;
          const double U = dPx * dRy - dPy * dRx;
          const double V = dqx * dRy - dqy * dRx;
          const bool a0 = s0 & split0, a1 = s1 & split1;
          const bool u_pos = U > 0.0, v_pos = V > 0.0;
          const bool f[4] = {(bool)(a0 & u_pos), (bool)(a0 & !u_pos & (V < 0.0)), (bool)(a1 & v_pos),
                             (bool)(a1 & !v_pos & (U < 0.0))};
          const double kk[4] = {U, -V, V, -U};
          offer<USER, 4>(b, f, kk, x, y, pos, pi[v], src);
          oh[v] = ((f[0] | (s0 & copy0)) ? 1u : 0u) | (f[1] ? 256u : 0u) | ((f[2] | (s1 & copy1)) ? 65536u : 0u) |
                  (f[3] ? 16777216u : 0u);
        }
      }
      // The classification is materialised in vector registers point by
      // point: otherwise the compiler keeps every point's lane masks alive in
      // scalar registers until the write loop and spills them.
      if constexpr (ARGMAX) {
        asm volatile("" : "+v"(m[0]), "+v"(m[1]));
      } else {
        asm volatile("" : "+v"(oh[v]));
      }
    }
    if constexpr (ARGMAX) {
      run1 += (uint32_t)__popc(m[0]);
      run2 += (uint32_t)__popc(m[1]);
      if (__ballot(bad) && lane == 0) A.req[req].err = 1u;
      bad = false;
    } else {
      write_onehot<BLOCK, PPT, NS, USER>(oh, cbeg, ccnt, cctr, px, py, pi, lo + tid - ibase, A.ox, A.oy, A.oi, s_cnt,
                                         s_base);
    }
  }
  if (run_seg != kNone) {
    flush_run<USER, NW>(src, A.part, run_slot, b[0], b[1], ibase, s_cand);
    if constexpr (FUSED) flush_run<USER, NW>(src, A.part2, run_slot, b[2], b[3], ibase, s_cand);
    if constexpr (ARGMAX) flush_counts<NW>(A.ctr + (size_t)run_seg * kCtrStride, run1, run2, s_cnt);
  }
}

// --------------------------------------------------------- block utilities

// Exclusive scan of N values per thread across a workgroup of BLOCK threads.
// TRAIL = false leaves out the closing barrier: the caller guarantees that
// every thread passes another barrier before s_w is written again.
template <int BLOCK, int N, bool TRAIL = true>
__device__ __forceinline__ void block_scan(const uint32_t (&v)[N], uint32_t (&excl)[N], uint32_t (&total)[N],
                                           uint32_t (*s_w)[BLOCK / 64]) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t inc[N];  // inclusive prefix within the wave (DPP row shifts and broadcasts)
#pragma unroll
  for (int j = 0; j < N; ++j) inc[j] = wave_scan_incl(v[j]);
  if (lane == 63) {
#pragma unroll
    for (int j = 0; j < N; ++j) s_w[j][w] = inc[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    uint32_t before = 0, all = 0;
    for (int i = 0; i < NW; ++i) {
      const uint32_t x = s_w[j][i];
      if (i < w) before += x;
      all += x;
    }
    excl[j] = before + inc[j] - v[j];
    total[j] = all;
  }
  if constexpr (TRAIL) __syncthreads();
}

// Best candidate over a workgroup; the result is valid in every thread.
template <int BLOCK>
__device__ __forceinline__ Cand block_best(Cand c, Cand* s_c) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  wave_best_fast(c);
  if (lane == 0) s_c[w] = c;
  __syncthreads();
  Cand r = s_c[0];
  for (int i = 1; i < NW; ++i)
    keep(r, s_c[i]);
  __syncthreads();
  return r;
}


// Visit records first, first + stride, ... below n with U loads in flight
// per thread (the records of a level were written by other compute units, so
// each load is a full memory round trip).
template <int U, typename Rec, typename F>
__device__ __forceinline__ void strided_visit(const Rec* rec, uint32_t first, uint32_t n, uint32_t stride, F&& f) {
  for (uint32_t k = first; k < n; k += U * stride) {
    Rec r[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const uint32_t kj = k + (uint32_t)j * stride;
      if (kj < n) r[j] = rec[kj];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (k + (uint32_t)j * stride < n) f(r[j]);
    }
  }
}

// ------------------------------------------------------------------ plans
//
// Each side of a partition step (a "child") becomes, by its size: nothing
// (no point), a leaf vertex (one point: Algorithm 1's base case), a finisher
// job (2 .. lds_limit points) or a segment of the next sweep level.  Every
// child with at least one point owns one node of the recursion tree, whose
// vertex is the child's farthest point.  A root (the top-level triangle
// (p, q, p) of a request) is always a job or a segment so that its points are
// read once and checked for non-finite values.

enum : uint32_t { kKindNone = 0, kKindLeaf = 1, kKindJob = 2, kKindSeg = 3 };

constexpr int kPlanBlock = 512;
constexpr int kPlanWaves = kPlanBlock / 64;
constexpr uint32_t kSerialRecs = 64;   // segments with more candidate records are reduced by one wave,
constexpr uint32_t kWaveRecs = 2048;   // and with more than this by the whole workgroup
constexpr uint32_t kSerialFill = 16;  // segments with more tiles get their tile map filled by the workgroup

__device__ __forceinline__ uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1u) / b; }

__device__ __forceinline__ uint32_t child_kind(uint32_t cnt, uint32_t lds_limit) {
  return cnt == 0u ? kKindNone : cnt == 1u ? kKindLeaf : cnt <= lds_limit ? kKindJob : kKindSeg;
}

template <int PB>
struct PlanSharedT {
  uint32_t scan[kPlanCounters][PB / 64];
  uint32_t nodes, jobs, segs, tiles, swept, jobpts, survivors;
  uint32_t pre[kPlanCounters];  // level planners: the totals of the rounds before this one
  uint32_t lb_fail;
  uint32_t nbig, nfill;
  uint32_t big[PB];
  uint32_t fill[2 * PB];  // up to two new segments per thread: id,
  uint32_t fill_t0[2 * PB];  // first tile
  uint32_t fill_nt[2 * PB];  // and tile count
};
using PlanShared = PlanSharedT<kPlanBlock>;

struct Tri {
  double ax, ay, rx, ry, bx, by;
};

// Offsets of this thread's children in the next level's tables.
struct EmitBase {
  uint32_t node, job, seg, tile;
};

template <int PB>
__device__ __forceinline__ EmitBase emit_scan(const uint32_t (&kind)[2], const uint32_t (&cnt)[2], uint32_t tile,
                                              PlanSharedT<PB>& S, uint32_t (&tot)[4], bool virt = false) {
  uint32_t v[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    v[0] += kind[k] != kKindNone;
    v[1] += kind[k] == kKindJob;
    v[2] += kind[k] == kKindSeg;
    v[3] += (kind[k] == kKindSeg && !virt) ? ceil_div(cnt[k], tile) : 0u;
  }
  uint32_t ex[4];
  block_scan<PB, 4>(v, ex, tot, S.scan);
  return EmitBase{S.nodes + ex[0], S.jobs + ex[1], S.segs + ex[2], S.tiles + ex[3]};
}

// Write one child (node, job or segment); advances the running offsets in e.
// A virtual segment (fused pass) gets no tiles: its candidates are written by
// the fused pass into the record slots of its root (vrec0, vrtiles, side).
struct Virt {
  bool on;
  uint32_t rec0, rtiles;
  unsigned long long* jctr_out;
};

template <int PB>
__device__ __forceinline__ int32_t emit_one(uint32_t kind, const Tri& tr, uint32_t ri, uint32_t beg, uint32_t cnt,
                                            uint32_t req, int32_t parent, uint32_t side, uint32_t src,
                                            uint32_t node_base, uint32_t tile, EmitBase& e, Node* nodes, Job* jobs,
                                            Seg* seg_out, unsigned long long* ctr_out, uint32_t* tile_seg_out,
                                            PlanSharedT<PB>& S, const Virt& vt, uint32_t* index_out,
                                            bool count_pts = true) {
  int32_t nid = -1;
  if (kind != kKindNone) {
    nid = (int32_t)(node_base + e.node++);
    Node nd;
    nd.vertex = ri;
    nd.c[0] = -1;
    nd.c[1] = -1;
    nd.size = kind == kKindLeaf ? 1u : 0u;
    nd.start = 0;
    nd.req = req;
    nd.list = kNone;
    nd.lbuf = 0;
    nodes[nid] = nd;
  }
  if (parent >= 0) nodes[parent].c[side] = nid;
  if (kind == kKindJob) {
    Job j;
    j.ax = tr.ax;
    j.ay = tr.ay;
    j.rx = tr.rx;
    j.ry = tr.ry;
    j.bx = tr.bx;
    j.by = tr.by;
    j.ri = ri;
    j.beg = beg;
    j.cnt = cnt;
    j.src = src;
    j.req = req;
    j.node = nid;
    j.ibase = src == kSrcUser ? beg : 0u;
    j.pad = 0;
    const uint32_t jid = e.job++;
    jobs[jid] = j;
    if (vt.on) vt.jctr_out[(size_t)jid * kCtrStride] = 0ull;
    *index_out = jid;
    if (count_pts) atomicAdd(&S.jobpts, cnt);
  } else if (kind == kKindSeg && vt.on) {
    const uint32_t sid = e.seg++;
    Seg sg;
    sg.ax = tr.ax;
    sg.ay = tr.ay;
    sg.rx = tr.rx;
    sg.ry = tr.ry;
    sg.bx = tr.bx;
    sg.by = tr.by;
    sg.beg = beg;
    sg.cnt = cnt;
    sg.tile0 = vt.rec0;
    sg.req = req;
    sg.node = nid;
    sg.ibase = 0u;
    sg.rtiles = vt.rtiles;
    sg.rside = side;
    seg_out[sid] = sg;
    ctr_out[(size_t)sid * kCtrStride] = 0ull;
    *index_out = sid;
    if (count_pts) atomicAdd(&S.swept, cnt);
  } else if (kind == kKindSeg) {
    const uint32_t sid = e.seg++;
    const uint32_t nt = ceil_div(cnt, tile);
    const uint32_t t0 = e.tile;
    e.tile += nt;
    *index_out = sid;
    Seg sg;
    sg.ax = tr.ax;
    sg.ay = tr.ay;
    sg.rx = tr.rx;
    sg.ry = tr.ry;
    sg.bx = tr.bx;
    sg.by = tr.by;
    sg.beg = beg;
    sg.cnt = cnt;
    sg.tile0 = t0;
    sg.req = req;
    sg.node = nid;
    sg.ibase = src == kSrcUser ? beg : 0u;
    sg.rtiles = 0u;
    sg.rside = 0u;
    seg_out[sid] = sg;
    ctr_out[(size_t)sid * kCtrStride] = 0ull;
    if (count_pts) atomicAdd(&S.swept, cnt);
    if (nt <= kSerialFill) {
      for (uint32_t i = 0; i < nt; ++i) tile_seg_out[t0 + i] = sid;
    } else {
      const uint32_t f = atomicAdd(&S.nfill, 1u);
      S.fill[f] = sid;
      S.fill_t0[f] = t0;
      S.fill_nt[f] = nt;
    }
  }
  return nid;
}

// Tile maps of the big new segments (a few: the whole workgroup over each
// one's tiles; many: one wave per segment), then running totals.
template <int PB, int NT = 4>
__device__ __forceinline__ void emit_finish(const uint32_t (&tot)[NT], uint32_t* tile_seg_out, PlanSharedT<PB>& S,
                                            bool running = true) {
  __syncthreads();
  const uint32_t nf = S.nfill;
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  if (nf <= PB / 64) {
    for (uint32_t f = 0; f < nf; ++f) {
      const uint32_t sid = S.fill[f], t0 = S.fill_t0[f], nt = S.fill_nt[f];
      for (uint32_t i = threadIdx.x; i < nt; i += PB) tile_seg_out[t0 + i] = sid;
    }
  } else {
    for (uint32_t f = w; f < nf; f += PB / 64) {
      const uint32_t sid = S.fill[f], t0 = S.fill_t0[f], nt = S.fill_nt[f];
      for (uint32_t i = lane; i < nt; i += 64u) tile_seg_out[t0 + i] = sid;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (running) {
      S.nodes += tot[0];
      S.jobs += tot[1];
      S.segs += tot[2];
      S.tiles += tot[3];
    }
    S.nfill = 0;
    S.nbig = 0;
  }
  __syncthreads();
}

template <int PB>
__device__ __forceinline__ void plan_init(PlanSharedT<PB>& S) {
  if (threadIdx.x == 0) {
    S.nodes = S.jobs = S.segs = S.tiles = S.swept = S.jobpts = S.survivors = 0;
    S.nbig = S.nfill = 0;
  }
  __syncthreads();
}

// The status record goes to the device ring (read by the next level's
// kernels) and, when host_out is set, straight to the host's pinned copy (read
// by the host after the event that follows this kernel), so no copy is
// enqueued per level.
__device__ __forceinline__ void put_status(const Status& st, Status* out, uint64_t* host_out, uint32_t tag) {
  *out = st;
  if (host_out) {
    const uint32_t v[kStatusWords] = {st.nseg, st.ntiles, st.njobs, st.nnodes, st.swept, st.jobpts, st.survivors,
                                      st.overflow};
    const uint64_t t = (uint64_t)tag << 32;
#pragma unroll
    for (int i = 0; i < kStatusWords; ++i)
      __hip_atomic_store(host_out + i, t | v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int PB>
__device__ __forceinline__ void plan_status(PlanSharedT<PB>& S, Status* out, uint64_t* host_out, uint32_t tag, uint32_t node_base,
                                            uint32_t* level_nodes, uint32_t ntiles) {
  if (threadIdx.x == 0) {
    *level_nodes = node_base + S.nodes;
    Status st;
    st.nseg = S.segs;
    st.ntiles = ntiles;
    st.njobs = S.jobs;
    st.nnodes = node_base + S.nodes;
    st.swept = S.swept;
    st.jobpts = S.jobpts;
    st.survivors = S.survivors;
    st.overflow = 0;
    put_status(st, out, host_out, tag);
  }
}

__device__ __forceinline__ void plan_overflow(Status* out, uint64_t* host_out, uint32_t tag, uint32_t node_base,
                                              uint32_t* level_nodes, BatchCounts* counts) {
  if (threadIdx.x == 0) {
    *level_nodes = node_base;
    counts->overflow = 1u;
    Status st{};
    st.nnodes = node_base;
    st.overflow = 1;
    put_status(st, out, host_out, tag);
  }
}

// The status of a level planned in rounds: t = nodes, jobs, segments, tiles,
// swept points, job points, survivors (the inclusive totals of the last round).
__device__ __forceinline__ void plan_status_totals(const uint32_t (&t)[kPlanCounters], Status* out, uint64_t* host_out, uint32_t tag,
                                                   uint32_t node_base, uint32_t* level_nodes, uint32_t ntiles) {
  if (threadIdx.x == 0) {
    *level_nodes = node_base + t[0];
    Status st;
    st.nseg = t[2];
    st.ntiles = ntiles;
    st.njobs = t[1];
    st.nnodes = node_base + t[0];
    st.swept = t[4];
    st.jobpts = t[5];
    st.survivors = t[6];
    st.overflow = 0;
    put_status(st, out, host_out, tag);
  }
}

// Look-back records are read and written with device-scope atomics: the
// planner workgroups of a launch may run on different XCDs.
__device__ __forceinline__ uint32_t ld_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// A round's own totals (flag 1) or its inclusive totals (flag 2); one thread.
__device__ __forceinline__ void round_publish(PlanRound* R, const uint32_t (&v)[kPlanCounters], bool incl) {
  uint32_t* dst = incl ? R->incl : R->agg;
#pragma unroll
  for (int i = 0; i < kPlanCounters; ++i) st_relaxed(&dst[i], v[i]);
  st_release(&R->flag, incl ? 2u : 1u);
}

// Waits of the look-back before it gives up (each a short sleep and one load
// per lane; a round's predecessor publishes within microseconds).
constexpr uint32_t kLookbackSpins = 1u << 20;

// The totals of rounds 0 .. r-1, by one whole wave: lane l looks at round
// r - 1 - l (64 rounds a step) and the sum runs down to the nearest round with
// inclusive totals.  Returns false if a round never published.
__device__ bool round_lookback(const PlanRound* R, uint32_t r, uint32_t (&pre)[kPlanCounters]) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int i = 0; i < kPlanCounters; ++i) pre[i] = 0u;
  int64_t top = (int64_t)r - 1;  // the round lane 0 looks at
  uint32_t spins = 0;
  while (top >= 0) {
    const int64_t j = top - (int64_t)lane;
    const uint32_t f = j >= 0 ? ld_acquire(&R[j].flag) : 2u;  // before round 0: the empty prefix
    const unsigned long long m2 = __ballot(f == 2u), m0 = __ballot(f == 0u);
    const uint32_t stop = m2 ? (uint32_t)__builtin_ctzll(m2) : 64u;
    const unsigned long long upto = stop >= 63u ? ~0ull : (2ull << stop) - 1ull;  // lanes 0 .. stop
    if (m0 & upto) {  // a round before the nearest complete one has not published
      if (++spins > kLookbackSpins) return false;
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
#pragma unroll
    for (int i = 0; i < kPlanCounters; ++i) {
      uint32_t v = 0u;
      if (j >= 0 && lane <= stop) v = lane < stop ? ld_relaxed(&R[j].agg[i]) : ld_relaxed(&R[j].incl[i]);
      pre[i] += wave_sum(v);
    }
    if (stop < 64u) break;
    top -= 64;
  }
  return true;
}

// Lexicographic extremes of partial records (y is present in the records).
struct Ext {
  double mnx, mny, mxx, mxy;
  uint32_t mni, mxi;
};

__device__ __forceinline__ void ext_merge(Ext& e, double mnx, double mny, uint32_t mni, double mxx, double mxy,
                                          uint32_t mxi) {
  if (mni != kNone &&
      (e.mni == kNone || mnx < e.mnx || (mnx == e.mnx && (mny < e.mny || (mny == e.mny && mni < e.mni))))) {
    e.mnx = mnx;
    e.mny = mny;
    e.mni = mni;
  }
  if (mxi != kNone &&
      (e.mxi == kNone || mxx > e.mxx || (mxx == e.mxx && (mxy > e.mxy || (mxy == e.mxy && mxi < e.mxi))))) {
    e.mxx = mxx;
    e.mxy = mxy;
    e.mxi = mxi;
  }
}

__device__ __forceinline__ Ext no_ext() { return Ext{0.0, 0.0, 0.0, 0.0, kNone, kNone}; }

__device__ __forceinline__ Ext wave_ext(Ext me) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    Ext o;
    o.mnx = __shfl_xor(me.mnx, m, 64);
    o.mny = __shfl_xor(me.mny, m, 64);
    o.mni = __shfl_xor(me.mni, m, 64);
    o.mxx = __shfl_xor(me.mxx, m, 64);
    o.mxy = __shfl_xor(me.mxy, m, 64);
    o.mxi = __shfl_xor(me.mxi, m, 64);
    ext_merge(me, o.mnx, o.mny, o.mni, o.mxx, o.mxy, o.mxi);
  }
  return me;
}

// Root level: p and q of every request, then the degenerate triangle (p, q, p)
// of Algorithm 1's top level as a job or a level-0 segment.
__global__ __launch_bounds__(kPlanBlock) void k_plan0(Plan0Args A) {
  __shared__ PlanShared S;
  __shared__ Ext s_res[kPlanBlock];
  __shared__ Ext s_w[kPlanWaves];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  plan_init(S);
  const uint32_t nreq = A.counts->nreq;
  if ((uint64_t)nreq > A.node_cap) {
    if (threadIdx.x == 0) A.level_nodes[0] = 0u;
    plan_overflow(A.st_out, A.st_host, A.st_tag, 0u, A.level_nodes + 1, A.counts);
    return;
  }
  for (uint32_t base = 0; base < nreq; base += kPlanBlock) {
    const uint32_t i = base + tid;
    const bool valid = i < nreq;
    Req rq{};
    Ext e = no_ext();
    bool big = false;
    if (valid) {
      rq = A.req[i];
      const uint32_t nt = ceil_div(rq.n, A.ext_tile);
      if (nt <= kSerialRecs) {
        strided_visit<4>(A.epart + rq.tile0, 0u, nt, 1u,
                         [&](const ExtPart& p) { ext_merge(e, p.minx, p.miny, p.mini, p.maxx, p.maxy, p.maxi); });
      } else {
        big = true;
        S.big[atomicAdd(&S.nbig, 1u)] = (uint32_t)tid;
      }
    }
    __syncthreads();
    const uint32_t nbig = S.nbig;
    for (uint32_t b = w; b < nbig; b += kPlanWaves) {  // one wave per big request
      const uint32_t owner = S.big[b];
      const uint32_t t0 = A.req[base + owner].tile0, nt = ceil_div(A.req[base + owner].n, A.ext_tile);
      if (nt > kWaveRecs) continue;
      Ext me = no_ext();
      strided_visit<4>(A.epart + t0, (uint32_t)lane, nt, 64u,
                       [&](const ExtPart& p) { ext_merge(me, p.minx, p.miny, p.mini, p.maxx, p.maxy, p.maxi); });
      me = wave_ext(me);
      if (lane == 0) s_res[owner] = me;
    }
    for (uint32_t b = 0; b < nbig; ++b) {  // the whole workgroup per huge request
      const uint32_t owner = S.big[b];
      const uint32_t t0 = A.req[base + owner].tile0, nt = ceil_div(A.req[base + owner].n, A.ext_tile);
      if (nt <= kWaveRecs) continue;
      Ext me = no_ext();
      strided_visit<4>(A.epart + t0, (uint32_t)tid, nt, (uint32_t)kPlanBlock,
                       [&](const ExtPart& p) { ext_merge(me, p.minx, p.miny, p.mini, p.maxx, p.maxy, p.maxi); });
      me = wave_ext(me);
      if (lane == 0) s_w[w] = me;
      __syncthreads();
      if (tid == 0) {
        Ext f = no_ext();
        for (int q = 0; q < kPlanWaves; ++q)
          ext_merge(f, s_w[q].mnx, s_w[q].mny, s_w[q].mni, s_w[q].mxx, s_w[q].mxy, s_w[q].mxi);
        s_res[owner] = f;
      }
      __syncthreads();
    }
    __syncthreads();
    if (big) e = s_res[tid];
    // A request that went through the octagon filter (above the LDS
    // threshold with the prefilter on; every request of interleaved input)
    // has its kept points at the front of its range of buffer A.
    uint32_t kind[2] = {kKindNone, kKindNone}, cnt[2] = {0, 0};
    const bool filt = valid && A.toff != nullptr && rq.n > A.filter_min;
    if (valid && rq.n > 0) {
      cnt[0] = filt ? A.toff[rq.tile0 + ceil_div(rq.n, A.ext_tile)] - A.toff[rq.tile0] : rq.n;
      kind[0] = cnt[0] <= A.lds_limit ? kKindJob : kKindSeg;
    }
    uint32_t tot[4];
    EmitBase eb = emit_scan(kind, cnt, A.tile, S, tot);
    if (valid) {
      int32_t nid = -1;
      if (rq.n > 0) {
        const Tri tr{e.mnx, e.mny, e.mxx, e.mxy, e.mnx, e.mny};
        const Virt nov{false, 0u, 0u, nullptr};
        uint32_t idx = 0;
        nid = emit_one(kind[0], tr, e.mxi, rq.off, cnt[0], i, -1, 0, filt ? kSrcBufA : kSrcUser, 0u, A.tile, eb,
                       A.nodes, A.jobs, A.seg_out, A.ctr_out, A.tile_seg_out, S, nov, &idx);
      }
      A.req[i].p = rq.n > 0 ? e.mni : 0u;
      A.req[i].q = rq.n > 0 ? e.mxi : 0u;
      A.req[i].root = nid;
    }
    emit_finish(tot, A.tile_seg_out, S);
  }
  if (threadIdx.x == 0) A.level_nodes[0] = 0u;
  plan_status(S, A.st_out, A.st_host, A.st_tag, 0u, A.level_nodes + 1, S.tiles);
  // the look-back records of the level-0 planner start cleared
  const uint32_t nclr = min(A.rounds_cap, ceil_div(S.segs, kPlanRoundMin) + 1u);
  for (uint32_t c = threadIdx.x; c < nclr; c += kPlanBlock) st_relaxed(&A.rounds_next[c].flag, 0u);
}

// One recursion level: reduce the counts and candidates of every segment,
// then lay out its two children (Algorithm 1: Hull(S1, a, r1, r) and
// Hull(S2, r, r2, b)).  The children's points already sit at the two ends of
// the segment's range in the output buffer of the sweep.
template <int PB>
struct PlanLds {
  PlanSharedT<PB> S;
  Cand res[PB][2];
  Cand c[PB / 64];
};

template <int PB>
__device__ void plan_level(const PlanArgs& A, PlanLds<PB>& L, uint32_t g, uint32_t P) {
  constexpr int NWP = PB / 64;
  PlanSharedT<PB>& S = L.S;
  Cand (*s_res)[2] = L.res;
  Cand* s_c = L.c;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  plan_init(S);
  const uint32_t nseg = A.st_in->nseg, node_base = A.st_in->nnodes;
  const uint32_t nrounds = ceil_div(nseg, PB);
  if ((uint64_t)node_base + 2ull * nseg > A.node_cap || nrounds > A.rounds_cap) {
    if (g == 0) plan_overflow(A.st_out, A.st_host, A.st_tag, node_base, A.level_nodes + A.level + 2u, A.counts);
    return;
  }
  if (nrounds == 0) {  // an empty level: the next is empty too
    if (g == 0) {
      const uint32_t zero[kPlanCounters] = {0, 0, 0, 0, 0, 0, 0};
      plan_status_totals(zero, A.st_out, A.st_host, A.st_tag, node_base, A.level_nodes + A.level + 2u,
                         A.fuse ? A.st_in->ntiles : 0u);
    }
    return;
  }
  const uint32_t G = A.sweep_grid;
  uint32_t fin[kPlanCounters];  // inclusive totals of the last round (its workgroup writes the status)
  // Rounds of PB segments, taken by the planner workgroups in turn; each
  // round's output offsets are the totals of the rounds before it (look-back).
  for (uint32_t rr = g; rr < nrounds; rr += P) {
    const uint32_t base = rr * PB;
    const uint32_t s = base + tid;
    const bool valid = s < nseg;
    uint32_t n1 = 0, n2 = 0, tile0 = 0, nrec = 0;
    Cand r1 = no_cand(), r2 = no_cand();
    bool big = false;
    if (valid) {
      const unsigned long long c = A.ctr[(size_t)s * kCtrStride];
      n1 = (uint32_t)c;
      n2 = (uint32_t)(c >> 32);
      tile0 = A.seg[s].tile0;
      const uint32_t rt = A.seg[s].rtiles;
      nrec = min(G, rt ? rt : ceil_div(A.seg[s].cnt, A.tile));
      const TilePart* part = A.seg[s].rside ? A.part2 : A.part;
      if (nrec <= kSerialRecs) {
        strided_visit<4>(part + tile0, 0u, nrec, 1u, [&](const TilePart& p) {
          keep(r1, p.c[0]);
          keep(r2, p.c[1]);
        });
      } else {
        big = true;
        S.big[atomicAdd(&S.nbig, 1u)] = (uint32_t)tid;
      }
    }
    __syncthreads();
    const uint32_t nbig = S.nbig;
    for (uint32_t b = w; b < nbig; b += NWP) {  // one wave per big segment
      const uint32_t owner = S.big[b];
      const Seg& so = A.seg[base + owner];
      const uint32_t t0 = so.tile0;
      const uint32_t nr = min(G, so.rtiles ? so.rtiles : ceil_div(so.cnt, A.tile));
      const TilePart* part = so.rside ? A.part2 : A.part;
      if (nr > kWaveRecs) continue;
      Cand m1 = no_cand(), m2 = no_cand();
      strided_visit<4>(part + t0, (uint32_t)lane, nr, 64u, [&](const TilePart& p) {
        keep(m1, p.c[0]);
        keep(m2, p.c[1]);
      });
      wave_best_fast(m1);
      wave_best_fast(m2);
      if (lane == 0) {
        s_res[owner][0] = m1;
        s_res[owner][1] = m2;
      }
    }
    for (uint32_t b = 0; b < nbig; ++b) {  // the whole workgroup per huge segment
      const uint32_t owner = S.big[b];
      const Seg& so = A.seg[base + owner];
      const uint32_t t0 = so.tile0;
      const uint32_t nr = min(G, so.rtiles ? so.rtiles : ceil_div(so.cnt, A.tile));
      const TilePart* part = so.rside ? A.part2 : A.part;
      if (nr <= kWaveRecs) continue;
      Cand m1 = no_cand(), m2 = no_cand();
      strided_visit<4>(part + t0, (uint32_t)tid, nr, (uint32_t)PB, [&](const TilePart& p) {
        keep(m1, p.c[0]);
        keep(m2, p.c[1]);
      });
      m1 = block_best<PB>(m1, s_c);
      m2 = block_best<PB>(m2, s_c);
      if (tid == 0) {
        s_res[owner][0] = m1;
        s_res[owner][1] = m2;
      }
    }
    __syncthreads();
    if (big) {
      r1 = s_res[tid][0];
      r2 = s_res[tid][1];
    }
    uint32_t kind[2] = {kKindNone, kKindNone}, cnt[2] = {n1, n2};
    if (valid) {
      kind[0] = child_kind(n1, A.lds_limit);
      kind[1] = child_kind(n2, A.lds_limit);
    }
    // this thread's share of the round's counts
    uint32_t v[kPlanCounters] = {0, 0, 0, 0, 0, 0, n1 + n2};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      v[0] += kind[k] != kKindNone;
      v[1] += kind[k] == kKindJob;
      v[2] += kind[k] == kKindSeg;
      v[3] += (kind[k] == kKindSeg && !A.fuse) ? ceil_div(cnt[k], A.tile) : 0u;
      v[4] += kind[k] == kKindSeg ? cnt[k] : 0u;
      v[5] += kind[k] == kKindJob ? cnt[k] : 0u;
    }
    uint32_t ex[kPlanCounters], tot[kPlanCounters];
    block_scan<PB, kPlanCounters>(v, ex, tot, S.scan);
    // publish the round's totals and find those of the rounds before it
    if (tid == 0) {
      round_publish(A.rounds + rr, tot, rr == 0);
      if (rr == 0) {
#pragma unroll
        for (int i = 0; i < kPlanCounters; ++i) S.pre[i] = 0u;
      }
    }
    if (rr > 0 && w == 0) {
      uint32_t pre[kPlanCounters];
      const bool ok = round_lookback(A.rounds, rr, pre);
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kPlanCounters; ++i) S.pre[i] = pre[i];
        S.lb_fail = ok ? 0u : 1u;
        if (ok) {
          uint32_t incl[kPlanCounters];
#pragma unroll
          for (int i = 0; i < kPlanCounters; ++i) incl[i] = pre[i] + tot[i];
          round_publish(A.rounds + rr, incl, true);
        }
      }
    }
    __syncthreads();
    if (rr > 0 && S.lb_fail) {  // a round never published (not expected): report an overflow
      plan_overflow(A.st_out, A.st_host, A.st_tag, node_base, A.level_nodes + A.level + 2u, A.counts);
      return;
    }
    uint32_t pre[kPlanCounters];
#pragma unroll
    for (int i = 0; i < kPlanCounters; ++i) {
      pre[i] = S.pre[i];
      fin[i] = pre[i] + tot[i];
    }
    EmitBase eb{pre[0] + ex[0], pre[1] + ex[1], pre[2] + ex[2], pre[3] + ex[3]};
    if (valid) {
      const Seg sg = A.seg[s];
      const uint32_t root_tiles = ceil_div(sg.cnt, A.tile);
      const Virt vt{A.fuse != 0, sg.tile0, root_tiles, A.jctr_out};
      const Tri t1{sg.ax, sg.ay, r1.x, r1.y, sg.rx, sg.ry};
      uint32_t i1 = 0, i2 = 0;
      emit_one(kind[0], t1, r1.i, sg.beg, n1, sg.req, sg.node, 0, A.out_buf, node_base, A.tile, eb, A.nodes, A.jobs,
               A.seg_out, A.ctr_out, A.tile_seg_out, S, vt, &i1, false);
      const Tri t2{sg.rx, sg.ry, r2.x, r2.y, sg.bx, sg.by};
      emit_one(kind[1], t2, r2.i, sg.beg + sg.cnt - n2, n2, sg.req, sg.node, 1, A.out_buf, node_base, A.tile, eb,
               A.nodes, A.jobs, A.seg_out, A.ctr_out, A.tile_seg_out, S, vt, &i2, false);
      if (A.fuse) {
        FusedRoot f;
        f.px = sg.ax;
        f.py = sg.ay;
        f.qx = sg.rx;
        f.qy = sg.ry;
        f.bx = sg.bx;
        f.by = sg.by;
        const Tri* tt[2] = {&t1, &t2};
        const uint32_t idx[2] = {i1, i2};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          f.rx[c] = tt[c]->rx;
          f.ry[c] = tt[c]->ry;
          f.kind[c] = kind[c] == kKindSeg ? kFuseSplit : kind[c] == kKindJob ? kFuseCopy : kFuseSkip;
          f.slot[c] = idx[c];
        }
        f.beg[0] = sg.beg;
        f.cnt[0] = n1;
        f.beg[1] = sg.beg + sg.cnt - n2;
        f.cnt[1] = n2;
        f.off = sg.beg;
        f.n = sg.cnt;
        f.tile0 = sg.tile0;
        f.req = sg.req;
        A.fr_out[s] = f;
      }
    }
    emit_finish(tot, A.tile_seg_out, S, false);
  }
  // The workgroup of the last round knows the level's totals: the status,
  // and the look-back records of the next level planner cleared.
  if ((nrounds - 1u) % P == g) {
    // The fused pass walks the roots' tiles again.
    plan_status_totals(fin, A.st_out, A.st_host, A.st_tag, node_base, A.level_nodes + A.level + 2u,
                       A.fuse ? A.st_in->ntiles : fin[3]);
    const uint32_t nclr = min(A.rounds_cap, ceil_div(fin[2], kPlanRoundMin) + 1u);
    for (uint32_t i = tid; i < nclr; i += PB) st_relaxed(&A.rounds_next[i].flag, 0u);
  }
}

// ------------------------------------------------------- k_finish_plan
//
// One workgroup runs Algorithm 1 to the end on a subproblem (a, r, b) of at
// most TMAX points, entirely in LDS, breadth-first: every level classifies
// all live points of all live sub-subproblems at once.  Points are addressed
// by a local id (< TMAX, plus three ids for a, b and r of the root); the live
// list holds (sub-subproblem << 16 | local id).  Each level:
//   1. classify every live point, take a slot in its child with an LDS atomic;
//   2. scan the child sizes: nodes, next sub-subproblems and their ranges;
//   3. scatter the points into the next live list (one-point children record
//      their only point as their vertex);
//   4. find the farthest point of every child with >= 2 points (one thread per
//      small child, one wave per large child);
//   5. create the nodes and the next level's sub-subproblems.
// The ordered vertex list (in-order over the recursion tree) is written over
// the job's own index range.  Persistent: workgroups loop over the level's jobs.

constexpr uint16_t kNone16 = 0xFFFFu;
constexpr uint32_t kSmallChild = 32;  // children up to this size are reduced by one thread

template <int BLOCK, int TMAX>
struct FinishShared {
  dbl2 lp[TMAX + 3];  // coordinates: the job's points, then a, b and r
  uint32_t lid[TMAX + 3];
  uint32_t ord[2][TMAX];
  uint16_t sa[2][TMAX / 2], sr[2][TMAX / 2], sb[2][TMAX / 2], snode[2][TMAX / 2];
  uint32_t ccnt[TMAX];
  unsigned long long cmax[TMAX];  // largest key of each child (bits of a positive double)
  uint32_t ctie[TMAX];            // points of each child that reach that key
  uint16_t cwin[TMAX], cnode[TMAX], cbase[TMAX], cmap[TMAX];
  uint16_t nv[TMAX], nc0[TMAX], nc1[TMAX], nsz[TMAX], nst[TMAX];
  uint16_t lvl[TMAX + 2];
  uint16_t bigc[TMAX / kSmallChild + 2];
  uint32_t scan[3][BLOCK / 64];
  uint32_t bad, nbigc, anytie;
};

template <int BLOCK, int TMAX>
__device__ void finish_job(const Job& job, const FinishArgs& A, FinishShared<BLOCK, TMAX>& S) {
  constexpr int NW = BLOCK / 64;
  constexpr int KP = (TMAX + BLOCK - 1) / BLOCK;  // live points per thread per level
  constexpr int KC = (TMAX + BLOCK - 1) / BLOCK;  // children per thread per level
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t cnt = job.cnt;
  const bool user = job.src == kSrcUser;
  // the caller's points: the request's own arrays (position ibase = its point 0),
  // or the arrays passed in (a single request read by global position)
  const bool own = user && A.req_arrays;
  const double* X = user ? (own ? A.req[job.req].x - job.ibase : A.ux) : A.bx[job.src];
  const double* Y = user ? (own ? A.req[job.req].y - job.ibase : A.uy) : A.by[job.src];
  const uint32_t* I = user ? nullptr : A.bi[job.src];
  uint32_t* out = A.bi[user ? 0 : job.src] + job.beg;

  if (tid == 0) S.bad = 0;
  __syncthreads();
  bool bad = false;
  for (uint32_t l = tid; l < cnt; l += BLOCK) {
    const uint32_t pos = job.beg + l;
    const double xv = X[pos], yv = Y[pos];
    S.lp[l] = d2(xv, yv);
    S.lid[l] = user ? pos - job.ibase : I[pos];
    S.ord[0][l] = l;
    if (user) bad |= !finite(xv) || !finite(yv);
  }
  if (bad) S.bad = 1;
  if (tid == 0) {
    S.lp[cnt] = d2(job.ax, job.ay);
    S.lp[cnt + 1] = d2(job.bx, job.by);
    S.lp[cnt + 2] = d2(job.rx, job.ry);
    S.lid[cnt + 2] = job.ri;
    S.sa[0][0] = (uint16_t)cnt;
    S.sb[0][0] = (uint16_t)(cnt + 1);
    S.sr[0][0] = (uint16_t)(cnt + 2);
    S.snode[0][0] = 0;
    S.nv[0] = (uint16_t)(cnt + 2);
    S.nc0[0] = kNone16;
    S.nc1[0] = kNone16;
    S.lvl[0] = 0;
    S.lvl[1] = 1;
    S.nbigc = 0;
    S.anytie = 0;
  }
  if (tid < 2) {  // the two children of the first level
    S.ccnt[tid] = 0;
    S.cmax[tid] = 0ull;
    S.ctie[tid] = 0;
  }
  __syncthreads();
  if (S.bad && tid == 0) A.req[job.req].err = 1u;

  // Level sizes, identical in every thread (the scans return totals to all).
  uint32_t nsub_next = 1, ntot_next = cnt, nnode = 1, nlvl = 1;
  int cb = 0;  // live list buffer / sub-subproblem table of this level
  // The child counters of a level start at zero: the level before cleared
  // them in step 5 (each thread the children it owns there), with the
  // barrier that ends that step.
  while (nsub_next > 0) {
    const uint32_t nsub = nsub_next, ntot = ntot_next, nch = 2u * nsub;
    // 1. classify; the key of a point in its child (the orientation value that
    //    put it there, > 0) also enters the child's maximum: for positive
    //    doubles the bit patterns order like the values.
    uint32_t chd[KP], slot[KP], pid[KP];
    unsigned long long kb[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const uint32_t e = tid + k * BLOCK;
      chd[k] = kNone;
      slot[k] = 0;
      pid[k] = 0;
      kb[k] = 0ull;
      if (e < ntot) {
        const uint32_t ent = S.ord[cb][e];
        const uint32_t s = ent >> 16, l = ent & 0xFFFFu;
        const uint32_t a = S.sa[cb][s], r = S.sr[cb][s], b = S.sb[cb][s];
        const dbl2 pu = S.lp[l], pa = S.lp[a], pr = S.lp[r];
        const double ux = pu.x, uy = pu.y;
        const double o1 = orient(pa.x, pa.y, pr.x, pr.y, ux, uy);
        uint32_t c = kNone;
        double key = 0.0;
        if (o1 > 0.0) {
          c = 2u * s;
          key = o1;
        } else {
          const dbl2 pb = S.lp[b];
          const double o2 = orient(pr.x, pr.y, pb.x, pb.y, ux, uy);
          if (o2 > 0.0) {
            c = 2u * s + 1u;
            key = o2;
          }
        }
        if (c != kNone) {
          slot[k] = atomicAdd(&S.ccnt[c], 1u);
          kb[k] = __builtin_bit_cast(unsigned long long, key);
          atomicMax(&S.cmax[c], kb[k]);
        }
        chd[k] = c;
        pid[k] = l;
      }
    }
    __syncthreads();
    // 2. scan child sizes (children are assigned to threads in contiguous runs)
    {
      uint32_t v[3] = {0, 0, 0};
      const uint32_t c0 = tid * KC;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const uint32_t c = c0 + k;
        if (c < nch) {
          const uint32_t n = S.ccnt[c];
          v[0] += n >= 1u;
          v[1] += n >= 2u;
          v[2] += n >= 2u ? n : 0u;
        }
      }
      uint32_t ex[3], tot[3];
      block_scan<BLOCK, 3, false>(v, ex, tot, S.scan);  // the barrier below closes it
      uint32_t en = nnode + ex[0], es = ex[1], ep = ex[2];
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const uint32_t c = c0 + k;
        if (c < nch) {
          const uint32_t n = S.ccnt[c];
          S.cnode[c] = n >= 1u ? (uint16_t)en : kNone16;
          S.cmap[c] = n >= 2u ? (uint16_t)es : kNone16;
          S.cbase[c] = (uint16_t)ep;
          if (n > kSmallChild) S.bigc[atomicAdd(&S.nbigc, 1u)] = (uint16_t)c;
          en += n >= 1u;
          es += n >= 2u;
          ep += n >= 2u ? n : 0u;
        }
      }
      nnode += tot[0];
      nsub_next = tot[1];
      ntot_next = tot[2];
    }
    __syncthreads();
    // 3. scatter; the point holding its child's largest key is the child's
    //    farthest point unless another point of the child has the same key
    //    (then the full order decides below).
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const uint32_t c = chd[k];
      if (c != kNone) {
        if (S.ccnt[c] >= 2u) {
          S.ord[cb ^ 1][S.cbase[c] + slot[k]] = ((uint32_t)S.cmap[c] << 16) | pid[k];
          if (kb[k] == S.cmax[c]) {
            if (atomicAdd(&S.ctie[c], 1u) == 0u)
              S.cwin[c] = (uint16_t)pid[k];
            else
              S.anytie = 1u;
          }
        } else {
          S.cwin[c] = (uint16_t)pid[k];
        }
      }
    }
    __syncthreads();
    // 4. children whose largest key is shared by several points: farthest
    //    point by the full order (key, then x, y, index)
    if (S.anytie) {
    for (uint32_t c = tid; c < nch; c += BLOCK) {
      const uint32_t n = S.ccnt[c];
      if (n < 2u || n > kSmallChild || S.ctie[c] < 2u) continue;
      const uint32_t s = c >> 1;
      const uint32_t ea = (c & 1u) ? S.sr[cb][s] : S.sa[cb][s];
      const uint32_t eb = (c & 1u) ? S.sb[cb][s] : S.sr[cb][s];
      const dbl2 pea = S.lp[ea], peb = S.lp[eb];
      const double ex0 = pea.x, ey0 = pea.y, ex1 = peb.x, ey1 = peb.y;
      Cand best = no_cand();
      const uint32_t b0 = S.cbase[c];
      for (uint32_t e = 0; e < n; ++e) {
        const uint32_t l = S.ord[cb ^ 1][b0 + e] & 0xFFFFu;
        const dbl2 pl = S.lp[l];
        const double kk = orient(ex0, ey0, ex1, ey1, pl.x, pl.y);
        Cand o;
        o.k = kk;
        o.x = pl.x;
        o.y = pl.y;
        o.i = S.lid[l];
        o.pad = l;
        keep(best, o);
      }
      S.cwin[c] = (uint16_t)best.pad;
    }
    const uint32_t nbigc = S.nbigc;
    for (uint32_t b = w; b < nbigc; b += NW) {
      const uint32_t c = S.bigc[b];
      if (S.ctie[c] < 2u) continue;
      const uint32_t n = S.ccnt[c];
      const uint32_t s = c >> 1;
      const uint32_t ea = (c & 1u) ? S.sr[cb][s] : S.sa[cb][s];
      const uint32_t eb = (c & 1u) ? S.sb[cb][s] : S.sr[cb][s];
      const dbl2 pea = S.lp[ea], peb = S.lp[eb];
      const double ex0 = pea.x, ey0 = pea.y, ex1 = peb.x, ey1 = peb.y;
      Cand best = no_cand();
      const uint32_t b0 = S.cbase[c];
      for (uint32_t e = lane; e < n; e += 64) {
        const uint32_t l = S.ord[cb ^ 1][b0 + e] & 0xFFFFu;
        const dbl2 pl = S.lp[l];
        const double kk = orient(ex0, ey0, ex1, ey1, pl.x, pl.y);
        Cand o;
        o.k = kk;
        o.x = pl.x;
        o.y = pl.y;
        o.i = S.lid[l];
        o.pad = l;
        keep(best, o);
      }
      wave_best(best);  // pad carries the winner's local id
      if (lane == 0) S.cwin[c] = (uint16_t)best.pad;
    }
    __syncthreads();
    }
    // 5. nodes and next sub-subproblems; each thread then clears the child
    //    counters it owns for the next level (no other thread reads them
    //    in this step)
    const uint32_t nclr = max(nch, 2u * nsub_next);
    if (tid == 0) {
      S.nbigc = 0;
      S.anytie = 0;
    }
    for (uint32_t c = tid; c < nclr; c += BLOCK) {
      if (c >= nch) {
        S.ccnt[c] = 0;
        S.cmax[c] = 0ull;
        S.ctie[c] = 0;
        continue;
      }
      const uint32_t n = S.ccnt[c];
      const uint32_t s = c >> 1, side = c & 1u;
      const uint32_t parent = S.snode[cb][s];
      const uint16_t v = S.cnode[c];
      if (side) {
        S.nc1[parent] = v;
      } else {
        S.nc0[parent] = v;
      }
      if (n >= 1u) {
        S.nv[v] = S.cwin[c];
        S.nc0[v] = kNone16;
        S.nc1[v] = kNone16;
      }
      if (n >= 2u) {
        const uint32_t ns = S.cmap[c];
        S.sa[cb ^ 1][ns] = side ? S.sr[cb][s] : S.sa[cb][s];
        S.sb[cb ^ 1][ns] = side ? S.sb[cb][s] : S.sr[cb][s];
        S.sr[cb ^ 1][ns] = S.cwin[c];
        S.snode[cb ^ 1][ns] = v;
      }
      S.ccnt[c] = 0;
      S.cmax[c] = 0ull;
      S.ctie[c] = 0;
    }
    nlvl += 1;
    if (tid == 0) S.lvl[nlvl] = (uint16_t)nnode;  // read after the loop
    __syncthreads();
    cb ^= 1;
  }
  // in-order positions: subtree sizes bottom-up, starts top-down
  for (int L = (int)nlvl - 1; L >= 0; --L) {
    for (uint32_t v = S.lvl[L] + tid; v < S.lvl[L + 1]; v += BLOCK) {
      const uint16_t c0 = S.nc0[v], c1 = S.nc1[v];
      S.nsz[v] = (uint16_t)(1u + (c0 != kNone16 ? S.nsz[c0] : 0u) + (c1 != kNone16 ? S.nsz[c1] : 0u));
    }
    __syncthreads();
  }
  if (tid == 0) S.nst[0] = 0;
  __syncthreads();
  for (uint32_t L = 0; L < nlvl; ++L) {
    for (uint32_t v = S.lvl[L] + tid; v < S.lvl[L + 1]; v += BLOCK) {
      const uint16_t c0 = S.nc0[v], c1 = S.nc1[v];
      const uint32_t pos = S.nst[v] + (c0 != kNone16 ? S.nsz[c0] : 0u);
      out[pos] = S.lid[S.nv[v]];
      if (c0 != kNone16) S.nst[c0] = S.nst[v];
      if (c1 != kNone16) S.nst[c1] = (uint16_t)(pos + 1u);
    }
    __syncthreads();
  }
  if (tid == 0) {
    Node* nd = A.nodes + job.node;
    nd->size = S.nsz[0];
    nd->list = job.beg;
    nd->lbuf = user ? 0u : job.src;
  }
  __syncthreads();  // LDS is reused by the next job
}

// One launch per level for the finisher and the planner: workgroups
// 0 .. planners-1 plan the next level while the others finish this level's
// small subproblems.
// They share no data: the planner reads the sweep's counters and records and
// writes the next level's tables (its jobs into the other of the two job
// buffers); the finisher reads this level's jobs and points and fills in the
// vertex lists of this level's job nodes.
template <int BLOCK, int TMAX>
constexpr size_t finish_plan_lds() {
  return sizeof(FinishShared<BLOCK, TMAX>) > sizeof(PlanLds<BLOCK>) ? sizeof(FinishShared<BLOCK, TMAX>)
                                                                    : sizeof(PlanLds<BLOCK>);
}

template <int BLOCK, int TMAX>
__global__ __launch_bounds__(BLOCK) void k_finish_plan(FinishArgs A, PlanArgs P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (blockIdx.x < P.planners) {
    plan_level<BLOCK>(P, *reinterpret_cast<PlanLds<BLOCK>*>(smem_raw), blockIdx.x, P.planners);
    return;
  }
  FinishShared<BLOCK, TMAX>& S = *reinterpret_cast<FinishShared<BLOCK, TMAX>*>(smem_raw);
  const uint32_t njobs = A.st->njobs;
  for (uint32_t j = blockIdx.x - P.planners; j < njobs; j += gridDim.x - P.planners) {
    const Job job = A.jobs[j];
    finish_job<BLOCK, TMAX>(job, A, S);
  }
}

// ------------------------------------------------------------- k_small
//
// A single request small enough for the LDS finisher, in one launch: the
// lexicographic extremes p and q by a workgroup reduction (the non-finite
// check on the way), then Algorithm 1 from the degenerate triangle (p, q, p)
// inside LDS exactly as a root job of the level loop, and the clockwise list
// [p] ++ finisher list written to the caller's output.

// (x, y, index) order: the lexicographic minimum, and the maximum of (x, y)
// with the lower index among equal points.
__device__ __forceinline__ bool small_before(double xa, double ya, uint32_t ia, double xb, double yb, uint32_t ib) {
  if (ib == kNone) return ia != kNone;
  if (ia == kNone) return false;
  if (xa != xb) return xa < xb;
  if (ya != yb) return ya < yb;
  return ia < ib;
}
__device__ __forceinline__ bool small_after(double xa, double ya, uint32_t ia, double xb, double yb, uint32_t ib) {
  if (ib == kNone) return ia != kNone;
  if (ia == kNone) return false;
  if (xa != xb) return xa > xb;
  if (ya != yb) return ya > yb;
  return ia < ib;
}

template <int BLOCK, int TMAX>
__global__ __launch_bounds__(BLOCK) void k_small(SmallArgs A) {
  constexpr int NW = BLOCK / 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FinishShared<BLOCK, TMAX>& S = *reinterpret_cast<FinishShared<BLOCK, TMAX>*>(smem_raw);
  __shared__ double s_mn[2][NW], s_mx[2][NW];
  __shared__ uint32_t s_mni[NW], s_mxi[NW], s_bad;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t n = A.n;
  double mnx = 0.0, mny = 0.0, mxx = 0.0, mxy = 0.0;
  uint32_t mni = kNone, mxi = kNone;
  bool bad = false;
  for (uint32_t i = tid; i < n; i += BLOCK) {
    const double xv = A.x[i], yv = A.y[i];
    bad |= !finite(xv) || !finite(yv);
    if (small_before(xv, yv, i, mnx, mny, mni)) {
      mnx = xv;
      mny = yv;
      mni = i;
    }
    if (small_after(xv, yv, i, mxx, mxy, mxi)) {
      mxx = xv;
      mxy = yv;
      mxi = i;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double ax = __shfl_xor(mnx, m, 64), ay = __shfl_xor(mny, m, 64);
    const uint32_t ai = __shfl_xor(mni, m, 64);
    if (small_before(ax, ay, ai, mnx, mny, mni)) {
      mnx = ax;
      mny = ay;
      mni = ai;
    }
    const double bx = __shfl_xor(mxx, m, 64), by = __shfl_xor(mxy, m, 64);
    const uint32_t bi = __shfl_xor(mxi, m, 64);
    if (small_after(bx, by, bi, mxx, mxy, mxi)) {
      mxx = bx;
      mxy = by;
      mxi = bi;
    }
  }
  if (tid == 0) s_bad = 0u;
  __syncthreads();
  if (bad) s_bad = 1u;
  if (lane == 0) {
    s_mn[0][w] = mnx;
    s_mn[1][w] = mny;
    s_mni[w] = mni;
    s_mx[0][w] = mxx;
    s_mx[1][w] = mxy;
    s_mxi[w] = mxi;
  }
  __syncthreads();
  for (int i = 0; i < NW; ++i) {
    if (small_before(s_mn[0][i], s_mn[1][i], s_mni[i], mnx, mny, mni)) {
      mnx = s_mn[0][i];
      mny = s_mn[1][i];
      mni = s_mni[i];
    }
    if (small_after(s_mx[0][i], s_mx[1][i], s_mxi[i], mxx, mxy, mxi)) {
      mxx = s_mx[0][i];
      mxy = s_mx[1][i];
      mxi = s_mxi[i];
    }
  }
  // every thread now holds the same p = mni and q = mxi (uniform branches)
  if (s_bad) {
    if (tid == 0) *A.out_count = kCountNonfinite;
    return;
  }
  if (n == 0u) {
    if (tid == 0) *A.out_count = 0;
    return;
  }
  if (mni == mxi) {  // every point is the same point
    if (tid == 0) {
      A.out_idx[0] = mni;
      *A.out_count = 1;
    }
    return;
  }
  Job job;
  job.ax = mnx;
  job.ay = mny;
  job.rx = mxx;
  job.ry = mxy;
  job.bx = mnx;
  job.by = mny;
  job.ri = mxi;
  job.beg = 0;
  job.cnt = n;
  job.src = kSrcUser;
  job.req = 0;
  job.node = 0;
  job.ibase = 0;
  job.pad = 0;
  FinishArgs fa{};
  fa.ux = A.x;
  fa.uy = A.y;
  fa.bi[0] = A.list;
  fa.bi[1] = A.list;
  fa.nodes = A.node;
  fa.req = A.req;
  finish_job<BLOCK, TMAX>(job, fa, S);  // ends with a workgroup barrier
  const uint32_t size = S.nsz[0];  // the list: Hull(S1) ++ [q] ++ Hull(S2)
  for (uint32_t i = tid; i < size; i += BLOCK) A.out_idx[1 + i] = A.list[i];
  if (tid == 0) {
    A.out_idx[0] = mni;
    *A.out_count = (int64_t)size + 1;
  }
}

// ------------------------------------------------------ octagon prefilter
//
// A variant of the method (Section 6's Akl-Toussaint heuristic) for requests
// above the LDS threshold:
//   k_octagon      per extremes tile: the lexicographic extremes (the record
//                  the plain extremes pass writes) and the minima and maxima of
//                  y, fl(x - y) and fl(x + y), lowest index among equal values;
//                  both coordinates are checked for NaN and infinity.
//   k_oct_plan     per request: the vertices v0 = min y, v1 = max fl(x - y),
//                  v2 = q, v3 = max fl(x + y), v4 = max y, v5 = min fl(x - y),
//                  v6 = p, v7 = min fl(x + y) (counter-clockwise) and the
//                  records of the eight edges.
//   k_filter       per extremes tile: the points not strictly inside all eight
//                  edges, compacted to the tile's own start in buffer B.
//   k_filter_scan  one workgroup: the prefix of the kept counts over all tiles.
//   k_compact      per extremes tile: its kept points moved to their place at
//                  the front of the request's range in buffer A.
// Coordinates are taken relative to the origin o = p (u' = fl(u - o)).  Edge
// i runs from a = v_i to b = v_(i+1 mod 8), (ex, ey) = fl(b - a), and a point
// u is strictly inside it when
//   L(u) = fl(fl(ex * u'.y) - fl(ey * u'.x)) > t = fl(L(a) + m),
//   m = max(2^-44 * fl(fl(|ex| + |ey|) * D), 2^-900),
// with D = fl(fl(q.x - p.x) + fl(max y - min y)).  L(u) - L(a) is the cross
// product of the edge with u - a; the rounding errors of L(u), L(a), t and of
// the edge direction stay below 10 units in the last place of
// (|ex| + |ey|) * D (and below 2^-1070 where products underflow), far under
// m, so a dropped point is strictly left of every edge in exact arithmetic:
// the closed octagon winds around it, so it lies strictly inside the hull and
// never matters to the hull.  Zero-length edges (repeated vertices) are
// skipped (t = -inf); if all eight have zero length, or a vertex is missing (a
// non-finite input, reported as such), nothing is dropped (t = +inf).  Every
// operation is one rounded binary64 operation in the order written (no
// contraction); per point and edge the test is two products, one difference
// and one comparison.

constexpr int kOctBlock = 256, kOctPPT = 8, kOctIter = 8;
static_assert(kOctBlock * kOctPPT * kOctIter == (int)kExtTile, "the prefilter shares the extremes tiling");
constexpr int kScanBlock = 1024;

// (v, i) takes (ov, oi) if that is smaller (larger), or equal at a lower index.
__device__ __forceinline__ void oct_lower(double& v, uint32_t& i, double ov, uint32_t oi) {
  if (oi != kNone && (i == kNone || ov < v || (ov == v && oi < i))) {
    v = ov;
    i = oi;
  }
}
__device__ __forceinline__ void oct_higher(double& v, uint32_t& i, double ov, uint32_t oi) {
  if (oi != kNone && (i == kNone || ov > v || (ov == v && oi < i))) {
    v = ov;
    i = oi;
  }
}

// Running extremes of one thread / wave / workgroup: the lexicographic pair
// and the three direction pairs (index kNone: none yet).
struct OctAcc {
  double lnx, lny, lxx, lxy;
  uint32_t lni, lxi;
  double mn[3], mx[3];
  uint32_t imn[3], imx[3];
};

__device__ __forceinline__ OctAcc oct_empty() {
  OctAcc a;
  a.lnx = a.lny = a.lxx = a.lxy = 0.0;
  a.lni = a.lxi = kNone;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a.mn[d] = a.mx[d] = 0.0;
    a.imn[d] = a.imx[d] = kNone;
  }
  return a;
}

__device__ __forceinline__ void oct_merge(OctAcc& a, const OctAcc& o) {
  if (small_before(o.lnx, o.lny, o.lni, a.lnx, a.lny, a.lni)) {
    a.lnx = o.lnx;
    a.lny = o.lny;
    a.lni = o.lni;
  }
  if (small_after(o.lxx, o.lxy, o.lxi, a.lxx, a.lxy, a.lxi)) {
    a.lxx = o.lxx;
    a.lxy = o.lxy;
    a.lxi = o.lxi;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    oct_lower(a.mn[d], a.imn[d], o.mn[d], o.imn[d]);
    oct_higher(a.mx[d], a.imx[d], o.mx[d], o.imx[d]);
  }
}

__device__ __forceinline__ OctAcc oct_shfl_xor(const OctAcc& a, int m) {
  OctAcc o;
  o.lnx = __shfl_xor(a.lnx, m, 64);
  o.lny = __shfl_xor(a.lny, m, 64);
  o.lni = __shfl_xor(a.lni, m, 64);
  o.lxx = __shfl_xor(a.lxx, m, 64);
  o.lxy = __shfl_xor(a.lxy, m, 64);
  o.lxi = __shfl_xor(a.lxi, m, 64);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o.mn[d] = __shfl_xor(a.mn[d], m, 64);
    o.mx[d] = __shfl_xor(a.mx[d], m, 64);
    o.imn[d] = __shfl_xor(a.imn[d], m, 64);
    o.imx[d] = __shfl_xor(a.imx[d], m, 64);
  }
  return o;
}

// Merge over the workgroup; the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ OctAcc oct_block(OctAcc a, OctAcc* s_w) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) oct_merge(a, oct_shfl_xor(a, m));
  if (lane == 0) s_w[w] = a;
  __syncthreads();
  if (tid == 0)
    for (int i = 1; i < NW; ++i) oct_merge(a, s_w[i]);
  return a;
}

template <int BLOCK, int PPT, int ITER, bool AOS>
__global__ __launch_bounds__(BLOCK) void k_octagon(OctArgs A) {
  constexpr uint32_t SUB = BLOCK * PPT;
  constexpr uint32_t TILE = SUB * ITER;
  __shared__ OctAcc s_w[BLOCK / 64];
  const uint32_t t = blockIdx.x;
  if (t >= A.counts->ext_tiles) return;
  const uint32_t r = A.tile_req ? A.tile_req[t] : 0u;
  const uint32_t off = A.req[r].off, n = A.req[r].n, tile0 = A.req[r].tile0;
  const uint32_t lo = off + (t - tile0) * TILE;
  const uint32_t hi = min(off + n, lo + TILE);
  const int tid = threadIdx.x, lane = tid & 63;

  // A thread visits its positions in increasing order, so strict comparisons
  // keep the lowest index among equal values.  Positions past the end read
  // NaN, which no comparison selects.
  double lnx = __builtin_inf(), lny = __builtin_inf(), lxx = -__builtin_inf(), lxy = -__builtin_inf();
  uint32_t lni = kNone, lxi = kNone;
  double mn[3], mx[3];
  uint32_t imn[3], imx[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mn[d] = __builtin_inf();
    mx[d] = -__builtin_inf();
    imn[d] = imx[d] = kNone;
  }
  bool bad = false;
  for (int it = 0; it < ITER; ++it) {
    const uint32_t slo = lo + (uint32_t)it * SUB;
    if (slo >= hi) break;  // uniform
    double xs[PPT], ys[PPT];
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      if constexpr (AOS) {
        const dbl2 p = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(A.xy) + min(pos, hi - 1u));
        xs[v] = pos < hi ? p.x : __builtin_nan("");
        ys[v] = pos < hi ? p.y : __builtin_nan("");
      } else {
        xs[v] = pos < hi ? __builtin_nontemporal_load(A.x + pos) : __builtin_nan("");
        ys[v] = pos < hi ? __builtin_nontemporal_load(A.y + pos) : __builtin_nan("");
      }
    }
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      const double x = xs[v], y = ys[v];
      bad |= (pos < hi) & !(finite(x) & finite(y));
      const bool lt = (x < lnx) | ((x == lnx) & (y < lny));
      const bool gt = (x > lxx) | ((x == lxx) & (y > lxy));
      lnx = lt ? x : lnx;
      lny = lt ? y : lny;
      lni = lt ? pos : lni;
      lxx = gt ? x : lxx;
      lxy = gt ? y : lxy;
      lxi = gt ? pos : lxi;
      const double val[3] = {y, x - y, x + y};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const bool l = val[d] < mn[d], g = val[d] > mx[d];
        mn[d] = l ? val[d] : mn[d];
        imn[d] = l ? pos : imn[d];
        mx[d] = g ? val[d] : mx[d];
        imx[d] = g ? pos : imx[d];
      }
    }
  }
  if (__ballot(bad) && lane == 0) A.req[r].err = 1u;
  OctAcc a;
  a.lnx = lnx;
  a.lny = lny;
  a.lni = lni;
  a.lxx = lxx;
  a.lxy = lxy;
  a.lxi = lxi;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a.mn[d] = mn[d];
    a.mx[d] = mx[d];
    a.imn[d] = imn[d];
    a.imx[d] = imx[d];
  }
  a = oct_block<BLOCK>(a, s_w);
  if (tid == 0) {
    ExtPart e;
    e.minx = a.lnx;
    e.miny = a.lny;
    e.maxx = a.lxx;
    e.maxy = a.lxy;
    e.mini = a.lni != kNone ? a.lni - off : kNone;
    e.maxi = a.lxi != kNone ? a.lxi - off : kNone;
    e.pad[0] = e.pad[1] = 0;
    A.part[t] = e;
    OctPart o;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      o.mn[d] = a.mn[d];
      o.mx[d] = a.mx[d];
      o.imn[d] = a.imn[d] != kNone ? a.imn[d] - off : kNone;
      o.imx[d] = a.imx[d] != kNone ? a.imx[d] - off : kNone;
    }
    A.opart[t] = o;
  }
}

// One workgroup per request: reduce the request's tile records (two in
// flight per thread), then the eight vertices and edge records (thread 0).
constexpr int kOctPlanBlock = 1024;

__device__ __forceinline__ OctAcc oct_record(const ExtPart& p, const OctPart& o) {
  OctAcc b;
  b.lnx = p.minx;
  b.lny = p.miny;
  b.lni = p.mini;
  b.lxx = p.maxx;
  b.lxy = p.maxy;
  b.lxi = p.maxi;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b.mn[d] = o.mn[d];
    b.mx[d] = o.mx[d];
    b.imn[d] = o.imn[d];
    b.imx[d] = o.imx[d];
  }
  return b;
}

__global__ __launch_bounds__(kOctPlanBlock) void k_oct_plan(FilterArgs A) {
  __shared__ OctAcc s_w[kOctPlanBlock / 64];
  const uint32_t r = blockIdx.x;
  if (r >= A.counts->nreq) return;
  const Req rq = A.req[r];
  OctEdges* E = A.oct + r;
  if (rq.n <= A.min_points) {
    if (threadIdx.x == 0) E->on = 0u;
    return;
  }
  const uint32_t nt = ceil_div(rq.n, kExtTile);
  OctAcc a = oct_empty();
  uint32_t k = threadIdx.x;
  for (; k + kOctPlanBlock < nt; k += 2 * kOctPlanBlock) {
    const ExtPart p0 = A.part[rq.tile0 + k], p1 = A.part[rq.tile0 + k + kOctPlanBlock];
    const OctPart o0 = A.opart[rq.tile0 + k], o1 = A.opart[rq.tile0 + k + kOctPlanBlock];
    oct_merge(a, oct_record(p0, o0));
    oct_merge(a, oct_record(p1, o1));
  }
  if (k < nt) oct_merge(a, oct_record(A.part[rq.tile0 + k], A.opart[rq.tile0 + k]));
  a = oct_block<kOctPlanBlock>(a, s_w);
  if (threadIdx.x != 0) return;
  const uint32_t v[8] = {a.imn[0], a.imx[1], a.lxi, a.imx[2], a.imx[0], a.imn[1], a.lni, a.imn[2]};
  bool missing = false;
  double vx[8], vy[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    missing |= v[i] == kNone;
    const uint32_t pos = v[i] == kNone ? rq.off : rq.off + v[i];
    vx[i] = A.xy ? A.xy[2 * (size_t)pos] : A.x[pos];
    vy[i] = A.xy ? A.xy[2 * (size_t)pos + 1] : A.y[pos];
  }
  const double D = (vx[2] - vx[6]) + (vy[4] - vy[0]);
  const double ox = vx[6], oy = vy[6];
  int edges = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int b = (i + 1) & 7;
    const double ex = vx[b] - vx[i];
    const double ey = vy[b] - vy[i];
    const double ay = vy[i] - oy;
    const double ax = vx[i] - ox;
    const double c1 = ex * ay;
    const double c2 = ey * ax;
    const double c = c1 - c2;
    const double s = fabs(ex) + fabs(ey);
    const double sd = s * D;
    const double m = fmax(0x1p-44 * sd, 0x1p-900);
    double t = c + m;
    if (ex == 0.0 && ey == 0.0) {
      t = -__builtin_inf();
    } else {
      ++edges;
    }
    E->ex[i] = ex;
    E->ey[i] = ey;
    E->t[i] = t;
  }
  const bool keep_all = edges == 0 || missing || rq.n <= A.drop_min;
  if (keep_all) {
#pragma unroll
    for (int i = 0; i < 8; ++i) E->t[i] = __builtin_inf();
  }
  E->keep_all = keep_all ? 1u : 0u;
  E->ox = ox;
  E->oy = oy;
  E->on = 1u;
}

// Loads of one sub-tile: positions past the end re-read the last point.
template <int BLOCK, int PPT, bool AOS>
__device__ __forceinline__ void filter_loads(const FilterArgs& A, uint32_t slo, uint32_t hi, double (&px)[PPT],
                                             double (&py)[PPT]) {
#pragma unroll
  for (int v = 0; v < PPT; ++v) {
    const uint32_t pc = min(slo + v * BLOCK + threadIdx.x, hi - 1u);
    if constexpr (AOS) {
      const dbl2 p = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(A.xy) + pc);
      px[v] = p.x;
      py[v] = p.y;
    } else {
      px[v] = __builtin_nontemporal_load(A.x + pc);
      py[v] = __builtin_nontemporal_load(A.y + pc);
    }
  }
}

template <int BLOCK, int PPT, int ITER, bool AOS>
__global__ __launch_bounds__(BLOCK) void k_filter(FilterArgs A) {
  constexpr uint32_t SUB = BLOCK * PPT;
  constexpr uint32_t TILE = SUB * ITER;
  constexpr int NW = BLOCK / 64;
  __shared__ uint32_t s_cnt[NW];
  const uint32_t t = blockIdx.x;
  if (t >= A.counts->ext_tiles) return;
  const uint32_t r = A.tile_req ? A.tile_req[t] : 0u;
  const uint32_t off = A.req[r].off, n = A.req[r].n, tile0 = A.req[r].tile0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (n <= A.min_points) {
    if (tid == 0) A.tcount[t] = 0u;
    return;
  }
  const uint32_t lo = off + (t - tile0) * TILE;
  const uint32_t hi = min(off + n, lo + TILE);
  const OctEdges* E = A.oct + r;
  if (uni(E->keep_all)) {
    // Nothing is dropped: every point goes straight to its own position in
    // buffer A (the kept-count prefix of the request's tiles is then the
    // identity, and the compaction skips the request).
    for (int it = 0; it < ITER; ++it) {
      const uint32_t slo = lo + (uint32_t)it * SUB;
      if (slo >= hi) break;  // uniform
      double px[PPT], py[PPT];
      filter_loads<BLOCK, PPT, AOS>(A, slo, hi, px, py);
#pragma unroll
      for (int v = 0; v < PPT; ++v) {
        const uint32_t pos = slo + v * BLOCK + tid;
        if (pos < hi) {
          A.cx[pos] = px[v];
          A.cy[pos] = py[v];
          A.ci[pos] = pos - off;
        }
      }
    }
    if (tid == 0) A.tcount[t] = hi - lo;
    return;
  }
  const double ox = uni(E->ox), oy = uni(E->oy);
  double eex[8], eey[8], et[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    eex[i] = uni(E->ex[i]);
    eey[i] = uni(E->ey[i]);
    et[i] = uni(E->t[i]);
  }
  uint32_t wpos = lo;  // next free position of the tile's staging range (uniform)
  for (int it = 0; it < ITER; ++it) {
    const uint32_t slo = lo + (uint32_t)it * SUB;
    if (slo >= hi) break;  // uniform
    double px[PPT], py[PPT];
    filter_loads<BLOCK, PPT, AOS>(A, slo, hi, px, py);
    uint32_t m = 0u;  // bit v: the thread's v-th point is kept
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const bool ok = slo + v * BLOCK + tid < hi;
      const double uy = py[v] - oy;
      const double ux = px[v] - ox;
      bool in = true;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double l1 = eex[i] * uy;
        const double l2 = eey[i] * ux;
        in &= (l1 - l2) > et[i];
      }
      m |= (uint32_t)(ok & !in) << v;
    }
    const uint32_t wc = wave_sum((uint32_t)__popc(m));
    if (lane == 0) s_cnt[w] = wc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t c = s_cnt[i];
      before += i < w ? c : 0u;
      all += c;
    }
    __syncthreads();  // s_cnt is rewritten by the next sub-tile
    uint32_t o = uni(wpos + before);
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const bool keepv = (m >> v) & 1u;
      const unsigned long long bal = __ballot(keepv);
      if (keepv) {
        const uint32_t dst = o + lane_rank(bal);
        A.sx[dst] = px[v];
        A.sy[dst] = py[v];
        A.si[dst] = slo + v * BLOCK + tid - off;
      }
      o += (uint32_t)__popcll(bal);
    }
    wpos += all;
  }
  if (tid == 0) A.tcount[t] = wpos - lo;
}

__global__ __launch_bounds__(kScanBlock) void k_filter_scan(FilterArgs A) {
  __shared__ uint32_t s_w[1][kScanBlock / 64];
  constexpr uint32_t PER = 4;
  const uint32_t T = A.counts->ext_tiles;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < T; base += kScanBlock * PER) {
    uint32_t c[PER], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const uint32_t i = base + threadIdx.x * PER + j;
      c[j] = i < T ? A.tcount[i] : 0u;
      sum += c[j];
    }
    const uint32_t v[1] = {sum};
    uint32_t ex[1], tot[1];
    block_scan<kScanBlock, 1>(v, ex, tot, s_w);
    uint32_t run = carry + ex[0];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const uint32_t i = base + threadIdx.x * PER + j;
      if (i < T) A.toff[i] = run;
      run += c[j];
    }
    carry += tot[0];
  }
  if (threadIdx.x == 0) A.toff[T] = carry;
}

__global__ __launch_bounds__(256) void k_compact(FilterArgs A) {
  const uint32_t t = blockIdx.x;
  if (t >= A.counts->ext_tiles) return;
  const uint32_t r = A.tile_req ? A.tile_req[t] : 0u;
  const uint32_t off = A.req[r].off, n = A.req[r].n, tile0 = A.req[r].tile0;
  if (n <= A.min_points || A.oct[r].keep_all) return;
  const uint32_t cnt = A.tcount[t];
  const uint32_t src = off + (t - tile0) * kExtTile;
  const uint32_t dst = off + (A.toff[t] - A.toff[tile0]);
  // four points per thread in flight: all loads, then all stores
  constexpr uint32_t U = 4;
  for (uint32_t base = 0; base < cnt; base += 256u * U) {
    double vx[U], vy[U];
    uint32_t vi[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t i = min(base + u * 256u + threadIdx.x, cnt - 1u);
      vx[u] = __builtin_nontemporal_load(A.sx + src + i);
      vy[u] = __builtin_nontemporal_load(A.sy + src + i);
      vi[u] = __builtin_nontemporal_load(A.si + src + i);
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t i = base + u * 256u + threadIdx.x;
      if (i < cnt) {
        A.cx[dst + i] = vx[u];
        A.cy[dst + i] = vy[u];
        A.ci[dst + i] = vi[u];
      }
    }
  }
}

// Interleaved input without the prefilter: x and y copied into workspace
// buffer A, which the whole plain path then reads as the caller's arrays
// (nothing writes buffer A's coordinates before level 2, after the last read
// of the caller's arrays).  k_ingest also records each extremes tile's
// lexicographic extremes (the plain extremes pass's record, with the
// non-finite check on both coordinates), so that pass is not run;
// k_deinterleave is the plain copy for the one-launch small path.
template <int BLOCK, int PPT, int ITER>
__global__ __launch_bounds__(BLOCK) void k_ingest(IngestArgs A) {
  constexpr uint32_t SUB = BLOCK * PPT;
  constexpr uint32_t TILE = SUB * ITER;
  __shared__ OctAcc s_w[BLOCK / 64];
  const uint32_t t = blockIdx.x;
  if (t >= A.counts->ext_tiles) return;
  const uint32_t r = A.tile_req ? A.tile_req[t] : 0u;
  const uint32_t off = A.req[r].off, n = A.req[r].n, tile0 = A.req[r].tile0;
  const uint32_t lo = off + (t - tile0) * TILE;
  const uint32_t hi = min(off + n, lo + TILE);
  const int tid = threadIdx.x, lane = tid & 63;
  double lnx = __builtin_inf(), lny = __builtin_inf(), lxx = -__builtin_inf(), lxy = -__builtin_inf();
  uint32_t lni = kNone, lxi = kNone;
  bool bad = false;
  for (int it = 0; it < ITER; ++it) {
    const uint32_t slo = lo + (uint32_t)it * SUB;
    if (slo >= hi) break;  // uniform
    double xs[PPT], ys[PPT];
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      const dbl2 p = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(A.xy) + min(pos, hi - 1u));
      xs[v] = pos < hi ? p.x : __builtin_nan("");
      ys[v] = pos < hi ? p.y : __builtin_nan("");
    }
#pragma unroll
    for (int v = 0; v < PPT; ++v) {
      const uint32_t pos = slo + v * BLOCK + tid;
      if (pos < hi) {
        A.x[pos] = xs[v];
        A.y[pos] = ys[v];
      }
      const double x = xs[v], y = ys[v];
      bad |= (pos < hi) & !(finite(x) & finite(y));
      const bool lt = (x < lnx) | ((x == lnx) & (y < lny));
      const bool gt = (x > lxx) | ((x == lxx) & (y > lxy));
      lnx = lt ? x : lnx;
      lny = lt ? y : lny;
      lni = lt ? pos : lni;
      lxx = gt ? x : lxx;
      lxy = gt ? y : lxy;
      lxi = gt ? pos : lxi;
    }
  }
  if (__ballot(bad) && lane == 0) A.req[r].err = 1u;
  OctAcc a = oct_empty();
  a.lnx = lnx;
  a.lny = lny;
  a.lni = lni;
  a.lxx = lxx;
  a.lxy = lxy;
  a.lxi = lxi;
  a = oct_block<BLOCK>(a, s_w);
  if (tid == 0) {
    ExtPart e;
    e.minx = a.lnx;
    e.miny = a.lny;
    e.maxx = a.lxx;
    e.maxy = a.lxy;
    e.mini = a.lni != kNone ? a.lni - off : kNone;
    e.maxi = a.lxi != kNone ? a.lxi - off : kNone;
    e.pad[0] = e.pad[1] = 0;
    A.part[t] = e;
  }
}

__global__ __launch_bounds__(256) void k_deinterleave(const double* __restrict__ xy, double* __restrict__ x,
                                                      double* __restrict__ y, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride) {
    const dbl2 p = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(xy) + i);
    x[i] = p.x;
    y[i] = p.y;
  }
}

// The orientation predicate on n triples, in the two forms the kernels use:
// orient() as the finisher and planners call it, and the sweeps' form that
// forms a - u and b - u first (the same rounded operations in the same order).
// out[2i] and out[2i+1] receive the two values of triple i.
__global__ __launch_bounds__(256) void k_orient(const double* __restrict__ abc, uint64_t n, double* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride) {
    const double* t = abc + 6 * i;
    const double ax = t[0], ay = t[1], bx = t[2], by = t[3], ux = t[4], uy = t[5];
    out[2 * i] = orient(ax, ay, bx, by, ux, uy);
    const double dax = ax - ux, day = ay - uy, dbx = bx - ux, dby = by - uy;
    out[2 * i + 1] = dax * dby - day * dbx;
  }
}

// ------------------------------------------------------------- k_assemble
//
// Clockwise order of every request: [p] ++ in-order(root), where the root's
// vertex is q and in-order(v) = in-order(S1 child) ++ [v] ++ in-order(S2
// child) (Algorithm 1's unions in order).  One workgroup: subtree sizes
// bottom-up level by level, then output positions top-down.  Subtrees
// finished in LDS already hold their ordered lists; k_copy_lists moves them.

constexpr int kAsmBlock = 1024;
constexpr int kAsmUnroll = 4;  // nodes per thread whose loads are in flight together

// A stream-ordered call whose level budget ended before the recursion did.
__device__ __forceinline__ bool assembly_incomplete(const AssembleArgs& A) {
  if (!A.last) return false;
  const Status st = *A.last;
  return st.nseg != 0u || st.njobs != 0u || st.overflow != 0u || A.counts->overflow != 0u;
}

__global__ __launch_bounds__(kAsmBlock) void k_assemble(AssembleArgs A) {
  const int tid = threadIdx.x;
  if (assembly_incomplete(A)) {
    for (uint32_t i = tid; i < A.counts->nreq; i += kAsmBlock) A.out_count[i] = kCountIncomplete;
    return;
  }
  // Each thread takes kAsmUnroll nodes of a level at a time, their loads
  // issued together: a node's children sit on the next level, which is done,
  // so the nodes of one level do not depend on each other.
  for (int L = (int)A.nlevels - 1; L >= 0; --L) {
    const uint32_t end = A.level_begin[L + 1];
    for (uint32_t v0 = A.level_begin[L] + tid; v0 < end; v0 += kAsmUnroll * kAsmBlock) {
      int32_t c[kAsmUnroll][2];
      bool act[kAsmUnroll];
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
        const uint32_t v = v0 + (uint32_t)j * kAsmBlock;
        act[j] = false;
        c[j][0] = c[j][1] = -1;
        if (v < end) {
          const Node nd = A.nodes[v];
          act[j] = nd.list == kNone;
          c[j][0] = nd.c[0];
          c[j][1] = nd.c[1];
        }
      }
      uint32_t sz[kAsmUnroll][2];
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
#pragma unroll
        for (int e = 0; e < 2; ++e) sz[j][e] = (act[j] && c[j][e] >= 0) ? A.nodes[c[j][e]].size : 0u;
      }
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
        if (act[j]) A.nodes[v0 + (uint32_t)j * kAsmBlock].size = 1u + sz[j][0] + sz[j][1];
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  const uint32_t nreq = A.counts->nreq;
  for (uint32_t i = tid; i < nreq; i += kAsmBlock) {
    const Req rq = A.req[i];
    if (rq.root >= 0) A.nodes[rq.root].start = 1u;
  }
  __syncthreads();
  for (uint32_t L = 0; L < A.nlevels; ++L) {
    const uint32_t end = A.level_begin[L + 1];
    for (uint32_t v0 = A.level_begin[L] + tid; v0 < end; v0 += kAsmUnroll * kAsmBlock) {
      Node nd[kAsmUnroll];
      bool act[kAsmUnroll];
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
        const uint32_t v = v0 + (uint32_t)j * kAsmBlock;
        act[j] = v < end;
        if (act[j]) nd[j] = A.nodes[v];
      }
      uint32_t off[kAsmUnroll], s0[kAsmUnroll];
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
        off[j] = 0u;
        s0[j] = 0u;
        if (act[j]) {
          const Req rq = A.req[nd[j].req];
          act[j] = !rq.err && rq.p != rq.q && nd[j].list == kNone;
          off[j] = rq.off;
          if (act[j] && nd[j].c[0] >= 0) s0[j] = A.nodes[nd[j].c[0]].size;
        }
      }
#pragma unroll
      for (int j = 0; j < kAsmUnroll; ++j) {
        if (!act[j]) continue;
        const uint32_t pos = nd[j].start + s0[j];
        A.out_idx[off[j] + pos] = (int64_t)nd[j].vertex;
        if (nd[j].c[0] >= 0) A.nodes[nd[j].c[0]].start = nd[j].start;
        if (nd[j].c[1] >= 0) A.nodes[nd[j].c[1]].start = pos + 1u;
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  for (uint32_t i = tid; i < nreq; i += kAsmBlock) {
    const Req rq = A.req[i];
    int64_t count;
    if (rq.err) {
      count = kCountNonfinite;
    } else if (rq.n == 0) {
      count = 0;
    } else if (rq.p == rq.q) {
      A.out_idx[rq.off] = (int64_t)rq.p;
      count = 1;
    } else {
      A.out_idx[rq.off] = (int64_t)rq.p;
      count = 1 + (int64_t)A.nodes[rq.root].size;
    }
    A.out_count[i] = count;
  }
}

// Copy the ordered lists of LDS-finished subtrees into place (one wave each).
__global__ __launch_bounds__(256) void k_copy_lists(AssembleArgs A) {
  if (assembly_incomplete(A)) return;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * 256u) >> 6;
  const uint32_t nnodes = A.level_begin[A.nlevels];
  for (uint32_t v = wave; v < nnodes; v += nwaves) {
    const Node nd = A.nodes[v];
    if (nd.list == kNone) continue;
    const Req rq = A.req[nd.req];
    if (rq.err || rq.p == rq.q) continue;
    const uint32_t* src = A.lists[nd.lbuf] + nd.list;
    int64_t* dst = A.out_idx + rq.off + nd.start;
    for (uint32_t e = lane; e < nd.size; e += 64) dst[e] = (int64_t)src[e];
  }
}

// --------------------------------------------------------- k_stream_scale
// STREAM "Scale" (out = s * in): the achievable-bandwidth yardstick and the
// known-size kernel that calibrates the byte counters of the profiler.
__global__ __launch_bounds__(256) void k_stream_scale(const double* __restrict__ in, double* __restrict__ out,
                                                        uint64_t n, double s) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride) out[i] = s * in[i];
}

// ------------------------------------------------------ k_gather / k_scatter
// Batching server: requests arrive as separate device arrays.  k_gather packs
// them into one batch (request i at [off_i, off_i + n_i) of the staging
// arrays); k_scatter copies each request's count and vertex list from the
// batch output to the caller's buffers.  One workgroup per chunk of at most
// kServeChunk points of one request, so a large request spreads over many
// workgroups and a small one costs one.
__global__ __launch_bounds__(256) void k_gather(const ServedReq* __restrict__ reqs, const ServedChunk* __restrict__ chunks,
                                                const uint32_t* __restrict__ nchunks, double* __restrict__ dx,
                                                double* __restrict__ dy) {
  if (blockIdx.x >= *nchunks) return;
  const ServedChunk c = chunks[blockIdx.x];
  const ServedReq r = reqs[c.req];
  const uint64_t m = min((uint64_t)kServeChunk, (uint64_t)r.n - c.beg);
  for (uint64_t j = threadIdx.x; j < m; j += 256) {
    dx[r.off + c.beg + j] = __builtin_nontemporal_load(r.x + c.beg + j);
    dy[r.off + c.beg + j] = __builtin_nontemporal_load(r.y + c.beg + j);
  }
}

__global__ __launch_bounds__(256) void k_scatter(const ServedReq* __restrict__ reqs, const ServedChunk* __restrict__ chunks,
                                                 const uint32_t* __restrict__ nchunks, const int64_t* __restrict__ idx,
                                                 const int64_t* __restrict__ counts) {
  if (blockIdx.x >= *nchunks) return;
  const ServedChunk c = chunks[blockIdx.x];
  const ServedReq r = reqs[c.req];
  const int64_t cnt = counts[c.req];
  if (c.beg == 0 && threadIdx.x == 0) *r.out_count = cnt;
  if (cnt <= (int64_t)c.beg) return;  // also a negative (error) count
  const uint64_t m = min((uint64_t)kServeChunk, (uint64_t)cnt - c.beg);
  for (uint64_t j = threadIdx.x; j < m; j += 256) r.out_idx[c.beg + j] = idx[r.off + c.beg + j];
}

// -------------------------------------------------------------- launchers

namespace {
template <int BLOCK, int PPT>
int sweep_one(const SweepArgs& a, int mode, uint32_t grid, hipStream_t st) {
  if (mode == kSweepArgmax) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepArgmax>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else if (mode == kSweepFused) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepFused>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else if (mode == kSweepArgmaxWs) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepArgmaxWs>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else if (mode == kSweepFusedWs) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepFusedWs>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else if (mode == kSweepArgmaxPair) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepArgmaxPair>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else if (mode == kSweepFusedPair) {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepFusedPair>), dim3(grid), dim3(BLOCK), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_sweep<BLOCK, PPT, kSweepLevel>), dim3(grid), dim3(BLOCK), 0, st, a);
  }
  return (int)hipGetLastError();
}

template <int BLOCK, int PPT, int MODE>
uint32_t sweep_occupancy_grid() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_sweep<BLOCK, PPT, MODE>, BLOCK, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 256;
  return (uint32_t)(per_cu * cus);
}

}  // namespace

bool sweep_shape_supported(int block, int ppt) {
  return (block == 256 && (ppt == 16 || ppt == 32)) || (block == 512 && (ppt == 8 || ppt == 16)) ||
         (block == 1024 && ppt == 8);
}

// Grid sizes are computed once per shape and cached (atomics: calls on
// several host threads may ask at the same time; they compute equal values).
uint32_t sweep_grid(int block, int ppt, int mode) {
  static std::atomic<uint32_t> cache[5][kSweepModes] = {};
  const int k = block == 256 ? (ppt == 16 ? 0 : 1) : block == 512 ? (ppt == 8 ? 2 : 3) : 4;
  uint32_t g = cache[k][mode].load(std::memory_order_relaxed);
  if (!g) {
#define VQH_GRID(K, B, P)                                                          \
  if (k == K)                                                                      \
    g = mode == kSweepArgmax     ? sweep_occupancy_grid<B, P, kSweepArgmax>()   \
        : mode == kSweepFused    ? sweep_occupancy_grid<B, P, kSweepFused>()    \
        : mode == kSweepArgmaxWs ? sweep_occupancy_grid<B, P, kSweepArgmaxWs>() \
        : mode == kSweepFusedWs  ? sweep_occupancy_grid<B, P, kSweepFusedWs>()  \
        : mode == kSweepArgmaxPair ? sweep_occupancy_grid<B, P, kSweepArgmaxPair>() \
        : mode == kSweepFusedPair  ? sweep_occupancy_grid<B, P, kSweepFusedPair>()  \
                                 : sweep_occupancy_grid<B, P, kSweepLevel>();
    VQH_GRID(0, 256, 16)
    VQH_GRID(1, 256, 32)
    VQH_GRID(2, 512, 8)
    VQH_GRID(3, 512, 16)
    VQH_GRID(4, 1024, 8)
#undef VQH_GRID
    cache[k][mode].store(g, std::memory_order_relaxed);
  }
  return g;
}

int launch_extremes(const ExtremesArgs& a, void* stream) {
  if (a.ntiles == 0) return 0;
  hipLaunchKernelGGL((k_extremes<kExtBlock, kExtPPT, kExtIter>), dim3(a.ntiles), dim3(kExtBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_sweep(const SweepArgs& a, int mode, int block, int ppt, uint32_t grid, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (block == 256 && ppt == 16) return sweep_one<256, 16>(a, mode, grid, st);
  if (block == 256 && ppt == 32) return sweep_one<256, 32>(a, mode, grid, st);
  if (block == 512 && ppt == 8) return sweep_one<512, 8>(a, mode, grid, st);
  if (block == 512 && ppt == 16) return sweep_one<512, 16>(a, mode, grid, st);
  if (block == 1024 && ppt == 8) return sweep_one<1024, 8>(a, mode, grid, st);
  return (int)hipErrorInvalidValue;
}

int launch_plan0(const Plan0Args& a, void* stream) {
  hipLaunchKernelGGL(k_plan0, dim3(1), dim3(kPlanBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

// LDS finisher + planner launches (below the sweep launchers).
namespace {

// Workgroup size of the LDS finisher per job capacity.  Jobs of up to 1024
// points take 512 threads too: two such workgroups share a CU (~78 KB of LDS
// each), and their 16 waves hide the finisher's LDS latency better than 8.
constexpr int kFinishBlock512 = 256, kFinishBlock1024 = 512, kFinishBlock2048 = 512;
static_assert(sizeof(FinishShared<kFinishBlock2048, 2048>) <= 160 * 1024, "the LDS finisher fits one CU's LDS");

template <int BLOCK, int TMAX>
int finish_attr() {
  static std::atomic<bool> done{false};  // set once (repeating the call is harmless)
  if (!done.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute((const void*)k_finish_plan<BLOCK, TMAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)finish_plan_lds<BLOCK, TMAX>());
    if (e != hipSuccess) return (int)e;
    done.store(true, std::memory_order_release);
  }
  return 0;
}

// Grid: the planner's workgroup plus as many finisher workgroups as fit.
template <int BLOCK, int TMAX>
int finish_plan_one(const FinishArgs& a, const PlanArgs& p, hipStream_t st) {
  int e = finish_attr<BLOCK, TMAX>();
  if (e) return e;
  const size_t lds = finish_plan_lds<BLOCK, TMAX>();
  hipLaunchKernelGGL((k_finish_plan<BLOCK, TMAX>), dim3(p.planners + finish_grid(TMAX)), dim3(BLOCK), lds, st, a, p);
  return (int)hipGetLastError();
}

template <int BLOCK, int TMAX>
uint32_t finish_occupancy_grid() {
  if (finish_attr<BLOCK, TMAX>() != 0) return 256;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_finish_plan<BLOCK, TMAX>, BLOCK,
                                                   finish_plan_lds<BLOCK, TMAX>()) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 256;
  return (uint32_t)(per_cu * cus);
}

}  // namespace

int finish_tmax_for(int lds_limit) { return lds_limit <= 512 ? 512 : lds_limit <= 1024 ? 1024 : 2048; }

uint32_t finish_grid(int tmax) {
  static std::atomic<uint32_t> cache[3] = {};
  const int k = tmax == 512 ? 0 : tmax == 1024 ? 1 : 2;
  uint32_t g = cache[k].load(std::memory_order_relaxed);
  if (!g) {
    if (k == 0) g = finish_occupancy_grid<kFinishBlock512, 512>();
    if (k == 1) g = finish_occupancy_grid<kFinishBlock1024, 1024>();
    if (k == 2) g = finish_occupancy_grid<kFinishBlock2048, 2048>();
    cache[k].store(g, std::memory_order_relaxed);
  }
  return g;
}

int launch_octagon(const OctArgs& a, void* stream) {
  if (a.ntiles == 0) return 0;
  if (a.xy) {
    hipLaunchKernelGGL((k_octagon<kOctBlock, kOctPPT, kOctIter, true>), dim3(a.ntiles), dim3(kOctBlock), 0,
                       (hipStream_t)stream, a);
  } else {
    hipLaunchKernelGGL((k_octagon<kOctBlock, kOctPPT, kOctIter, false>), dim3(a.ntiles), dim3(kOctBlock), 0,
                       (hipStream_t)stream, a);
  }
  return (int)hipGetLastError();
}

int launch_oct_plan(const FilterArgs& a, uint32_t nreq, void* stream) {
  if (nreq == 0) return 0;
  hipLaunchKernelGGL(k_oct_plan, dim3(nreq), dim3(kOctPlanBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_filter(const FilterArgs& a, void* stream) {
  if (a.ntiles == 0) return 0;
  if (a.xy) {
    hipLaunchKernelGGL((k_filter<kOctBlock, kOctPPT, kOctIter, true>), dim3(a.ntiles), dim3(kOctBlock), 0,
                       (hipStream_t)stream, a);
  } else {
    hipLaunchKernelGGL((k_filter<kOctBlock, kOctPPT, kOctIter, false>), dim3(a.ntiles), dim3(kOctBlock), 0,
                       (hipStream_t)stream, a);
  }
  return (int)hipGetLastError();
}

int launch_filter_scan(const FilterArgs& a, void* stream) {
  hipLaunchKernelGGL(k_filter_scan, dim3(1), dim3(kScanBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_compact(const FilterArgs& a, void* stream) {
  if (a.ntiles == 0) return 0;
  hipLaunchKernelGGL(k_compact, dim3(a.ntiles), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_ingest(const IngestArgs& a, void* stream) {
  if (a.ntiles == 0) return 0;
  hipLaunchKernelGGL((k_ingest<kOctBlock, kOctPPT, kOctIter>), dim3(a.ntiles), dim3(kOctBlock), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_orient(const double* abc, uint64_t n, double* out, void* stream) {
  if (n == 0) return 0;
  const uint64_t blocks = std::min<uint64_t>((n + 255u) / 256u, 256u * 32u);
  hipLaunchKernelGGL(k_orient, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, abc, n, out);
  return (int)hipGetLastError();
}

int launch_deinterleave(const double* xy, double* x, double* y, uint64_t n, void* stream) {
  if (n == 0) return 0;
  const uint64_t blocks = std::min<uint64_t>((n + 255u) / 256u, 256u * 32u);
  hipLaunchKernelGGL(k_deinterleave, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, xy, x, y, n);
  return (int)hipGetLastError();
}

int launch_finish_plan(const FinishArgs& a, const PlanArgs& p, int tmax, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (tmax == 512) return finish_plan_one<kFinishBlock512, 512>(a, p, st);
  if (tmax == 1024) return finish_plan_one<kFinishBlock1024, 1024>(a, p, st);
  if (tmax == 2048) return finish_plan_one<kFinishBlock2048, 2048>(a, p, st);
  return (int)hipErrorInvalidValue;
}

template <int BLOCK, int TMAX>
int small_one(const SmallArgs& a, hipStream_t st) {
  static std::atomic<bool> done{false};  // set once (repeating the call is harmless)
  const size_t lds = sizeof(FinishShared<BLOCK, TMAX>);
  if (!done.load(std::memory_order_acquire)) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_small<BLOCK, TMAX>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    done.store(true, std::memory_order_release);
  }
  hipLaunchKernelGGL((k_small<BLOCK, TMAX>), dim3(1), dim3(BLOCK), lds, st, a);
  return (int)hipGetLastError();
}

int launch_small(const SmallArgs& a, int tmax, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (a.n > (uint32_t)tmax) return (int)hipErrorInvalidValue;
  if (tmax == 512) return small_one<kFinishBlock512, 512>(a, st);
  if (tmax == 1024) return small_one<kFinishBlock1024, 1024>(a, st);
  if (tmax == 2048) return small_one<kFinishBlock2048, 2048>(a, st);
  return (int)hipErrorInvalidValue;
}

int launch_stream_scale(const double* in, double* out, uint64_t n, double s, void* stream) {
  if (n == 0) return 0;
  const uint64_t blocks = std::min<uint64_t>((n + 255u) / 256u, 2048u);
  hipLaunchKernelGGL(k_stream_scale, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, in, out, n, s);
  return (int)hipGetLastError();
}

int launch_assemble(const AssembleArgs& a, void* stream) {
  hipLaunchKernelGGL(k_assemble, dim3(1), dim3(kAsmBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_copy_lists(const AssembleArgs& a, void* stream) {
  if (a.max_nodes == 0) return 0;
  const uint32_t waves = a.max_nodes < 65536u ? a.max_nodes : 65536u;
  hipLaunchKernelGGL(k_copy_lists, dim3((waves + 3u) / 4u), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_gather(const ServedReq* reqs, const ServedChunk* chunks, const uint32_t* nchunks, uint32_t grid, double* dx,
                  double* dy, void* stream) {
  if (grid == 0) return 0;
  hipLaunchKernelGGL(k_gather, dim3(grid), dim3(256), 0, (hipStream_t)stream, reqs, chunks, nchunks, dx, dy);
  return (int)hipGetLastError();
}

int launch_scatter(const ServedReq* reqs, const ServedChunk* chunks, const uint32_t* nchunks, uint32_t grid,
                   const int64_t* idx, const int64_t* counts, void* stream) {
  if (grid == 0) return 0;
  hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, (hipStream_t)stream, reqs, chunks, nchunks, idx, counts);
  return (int)hipGetLastError();
}

}  // namespace vqh
