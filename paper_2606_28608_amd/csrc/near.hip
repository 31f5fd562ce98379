// Near field: free-space DMK on the extended root grid with the root-level
// W_0 step omitted (Section 3.5, Algorithm 1 near-field step).
//
// Kernel split per level l (box side h_l = r_c / 2^l), eq:tele / eq:W0hat:
//   G - W_0 = sum_{l < L} D_l + R_L,
// D_l is exchanged as plane waves between colleague boxes that both have
// children; every target leaf sums the residual R directly over its list
// (built in tree.hip).  Plane waves of level l have period 3 h_l, modes
// k_j = 2 pi j / (3 h_l), |j_a| <= J, and carry D_l's Fourier multiplier
// divided by the period volume.  Boxes represent their sources by proxy
// charges on a p^d tensor Chebyshev grid, and their incoming field by proxy
// potentials on the same grid.
#include <array>

#include <rocblas/rocblas.h>

#include "internal.h"
#include "lagrange.h"

namespace pdmk {

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }
constexpr double kInv4Pi = 0.07957747154594767;
constexpr double kInv2Pi = 0.15915494309189535;

// ------------------------------------------------------------- residual sums
// slot pairs of the residual statistics (a power of two, at least 64) and of
// the colleague translation's counters (64)
constexpr int kStatSlots = 1024;
constexpr int kTransSlots = 64;

// out[0], out[1] = (add: +=) sums of nslots slot pairs (one wave; nslots a
// multiple of 64)
__global__ __launch_bounds__(64) void k_fold_stats(const unsigned long long* __restrict__ slots,
                                                   int nslots, unsigned long long* __restrict__ out,
                                                   int add) {
  unsigned long long a = 0, b = 0;
  for (int i = threadIdx.x; i < nslots; i += 64) {
    a += slots[2 * i];
    b += slots[2 * i + 1];
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    a += __shfl_xor(a, m);
    b += __shfl_xor(b, m);
  }
  if (threadIdx.x == 0) {
    out[0] = add ? out[0] + a : a;
    out[1] = add ? out[1] + b : b;
  }
}

// One 64-lane block per target leaf.  The block walks the concatenated source
// ranges of the leaf's list in tiles of 64 staged in LDS (each slot carries
// its own support h of the residual level), so short ranges do not leave
// tiles half empty.  Leaves with few targets split each tile over S lanes per
// target (S = 1, 2, 4, 8) and reduce across those lanes at the end.  The pair
// kernel is evaluated without branches and masked outside its support.
// 1/sqrt(x) in FP64: the hardware estimate (measured on gfx950: relative
// error below 2^-24) refined by NR Newton steps y <- y (3/2 - x y^2 / 2); one
// step leaves a relative error below 1e-14, two reach full precision.
template <int NR>
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
#pragma unroll
  for (int k = 0; k < NR; ++k) y = y * fma(-hx * y, y, 1.5);
  return y;
}
template <int NR>
__device__ inline double rsqrt_r(double x) { return rsqrt_f64<NR>(x); }
template <int NR>
__device__ inline float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double log_r(double x) { return log(x); }
__device__ inline float log_r(float x) { return __logf(x); }

// Real = double: FP64 throughout.  Real = float: the series, rsqrt and the
// sums over one tile of 64 sources in FP32, FP64 across tiles.
// q_s R(|x - y_s|) (and its gradient) for one pair, with R_h of eq:pswf_split:
// 3D 1/r - E(r^2/h^2)/h, 2D -log(r/h) + F2(r^2/h^2) (both without the 1/(4 pi),
// 1/(2 pi) factors), zero outside the support r < h and for the pair r = 0.
// Offsets and r^2 are formed in FP64 (an FP32 offset would lose u * h / r of r
// for the close pairs of a coarse leaf).  The series are monomials in
// u = 2 s - 1 = r^2 (2 / h^2) - 1, evaluated by Horner's rule.  A source slot
// carries (q, 1/h, 2/h^2) in Real.
template <class Real> struct SlotQ;
template <> struct SlotQ<float> { using T = float4; };
template <> struct SlotQ<double> { using T = double4; };
// target of a staged slot, kept in the unused fourth component of its charge
// vector (-1: none)
__device__ inline int slot_tg(const float4& w) { return __float_as_int(w.w); }
__device__ inline int slot_tg(const double4& w) { return (int)w.w; }
__device__ inline void set_slot_tg(float4& w, int tg) { w.w = __int_as_float(tg); }
__device__ inline void set_slot_tg(double4& w, int tg) { w.w = (double)tg; }

// SYM: also the pair's term for the source end, q_t R (q_t = qa, the charge
// of the target as a source), in *as (zero outside the support).
template <int D, int NE, bool GRAD, class Real, int NR, bool SYM = false>
__device__ inline void residual_pair(const double* x, const double4& sv,
                                     const typename SlotQ<Real>::T& sq, const Real* ec,
                                     const Real* edc, Real& acc, Real* g, int& nin,
                                     Real qa = 0, Real* as = nullptr) {
  static_assert(!(SYM && GRAD), "pairs evaluated once carry no gradients");
  if (SYM) *as = 0;
  double dd[3];
  dd[0] = x[0] - sv.x;
  dd[1] = x[1] - sv.y;
  dd[2] = D == 3 ? x[2] - sv.z : 0.0;
  double r2d = dd[0] * dd[0];
  r2d = fma(dd[1], dd[1], r2d);
  if (D == 3) r2d = fma(dd[2], dd[2], r2d);
  const bool in = r2d < sv.w && r2d > 0.0;   // sv.w = h^2 of the source's level
  // pairs inside the support, counted for the whole wave on the scalar unit
  // (every lane of the wave executes this line)
  {
    // (a ballot of each comparison maps onto its lane mask directly)
    const int c = __builtin_amdgcn_readfirstlane((int)__popcll(
        __builtin_amdgcn_ballot_w64(r2d < sv.w) & __builtin_amdgcn_ballot_w64(r2d > 0.0)));
    int u = __builtin_amdgcn_readfirstlane(nin);
    asm volatile("s_add_i32 %0, %0, %1" : "+s"(u) : "s"(c) : "scc");
    nin = u;
  }
  if (in) {
    const Real r2 = (Real)r2d;
    const Real qs = sq.x, ih = sq.y, ihh = sq.z;
    const Real u = fma(r2, ihh, (Real)-1);
    Real F = ec[NE - 1];
#pragma unroll
    for (int m = NE - 2; m >= 0; --m) F = fma(F, u, ec[m]);
    Real Fd = 0;
    if (GRAD) {
      Fd = edc[NE - 1];
#pragma unroll
      for (int m = NE - 2; m >= 0; --m) Fd = fma(Fd, u, edc[m]);
    }
    if (D == 3) {
      const Real ir = rsqrt_r<NR>(r2);
      const Real rv = fma(-F, ih, ir);
      acc = fma(qs, rv, acc);
      if (SYM) *as = qa * rv;
      if (GRAD) {
        const Real dx[3] = {(Real)dd[0], (Real)dd[1], (Real)dd[2]};
        const Real f = qs * (-ir * ir * ir - ihh * Fd * ih);
        for (int a = 0; a < D; ++a) g[a] = fma(f, dx[a], g[a]);
      }
    } else {
      const Real sgr = (Real)0.5 * r2 * ihh;   // s = r^2 / h^2
      const Real rv = (Real)-0.5 * log_r(sgr) + F;
      acc = fma(qs, rv, acc);
      if (SYM) *as = qa * rv;
      if (GRAD) {
        const Real dx[3] = {(Real)dd[0], (Real)dd[1], (Real)0};
        const Real f = qs * (-(Real)1 / r2 + ihh * Fd);
        for (int a = 0; a < D; ++a) g[a] = fma(f, dx[a], g[a]);
      }
    }
  }
}

// Cursor over the concatenated source list of one target leaf: each lane owns
// one slot of the current 64-slot tile (entry ee, offset oo inside it).
// Only positions before `end` (a segment boundary) are valid.
struct ListCursor {
  int ee, le, oo, rem;
  int4 en;
  __device__ void init(const int4* __restrict__ list, int lb, int le_, int slot, int end) {
    ee = lb;
    le = le_;
    oo = slot;
    rem = end - slot;
    en = ee < le ? list[ee] : make_int4(0, 0, 0, 0);
    walk(list);
  }
  __device__ void walk(const int4* __restrict__ list) {
    while (ee < le && oo >= en.y - en.x) {
      oo -= en.y - en.x;
      ++ee;
      if (ee < le) en = list[ee];
    }
  }
  __device__ void advance(const int4* __restrict__ list) {
    oo += 64;
    rem -= 64;
    walk(list);
  }
  __device__ bool valid() const { return ee < le && rem > 0; }
};

// Pairs evaluated once (targets = sources): the target leaf's own source
// range [sb, se) and the map from sorted images to sorted targets.
struct SymInfo {
  const int* itrg;
  int sb, se;
};

template <class Real>
struct SourceSlot {
  double4 v;                   // (offset, h^2)
  typename SlotQ<Real>::T w;   // (q, 1/h, 2/h^2, target of the source end: slot_tg)
  int tg;                      // SYM: target that also receives the pair (-1: none)
  bool live;                   // within h + rho of the pass's target centre
  // Source offset from the target leaf centre (formed in FP64) with the support
  // h^2 of its residual level in v.w, and (q, 1/h, 2/h^2, tg); slots past the list
  // end never interact (h^2 = 0).  live: the source can reach a target of the
  // pass, whose targets lie within rho of cc (|y - cc| < h + rho).
  // SYM: a source that is a point of the cell and a target of a later leaf
  // (in source order) receives the pair's term too (tg), also through a
  // virtual colleague's shift (its mirror entry has the opposite shift); one
  // of an earlier leaf is dropped (that leaf adds the pair to both ends);
  // image copies and the leaf's own sources are summed one way.
  template <bool SYM>
  __device__ void fetch(const ListCursor& c, const KParams& kp, const double* __restrict__ sx,
                        const double* __restrict__ sq, int64_t nimg, const double* cT, int D,
                        const double* cc, double rho, const SymInfo& si) {
    tg = -1;
    if (c.valid()) {
      const int sidx = c.en.x + c.oo;
      bool drop = false;
      if (SYM) {
        const int it = si.itrg[sidx];
        if (it >= 0) {
          if (sidx < si.sb) drop = true;
          else if (sidx >= si.se) tg = it;
        }
      }
      v.x = sx[sidx] - cT[0];
      v.y = sx[nimg + sidx] - cT[1];
      v.z = D == 3 ? sx[2 * nimg + sidx] - cT[2] : 0.0;
      if (c.en.w) {
        // a virtual image (rem:cube): the source shifted by L n
        int t = c.en.w - 1;
        double sh[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) {
          const double n = (double)(t % 3 - 1);
          t /= 3;
          for (int b = 0; b <= a; ++b) sh[b] = fma(kp.L[b + D * a], n, sh[b]);
        }
        v.x += sh[0];
        v.y += sh[1];
        v.z += sh[2];
      }
      // h = r_c 2^-z and 1/h = (1/r_c) 2^z (power-of-two scalings: exact)
      const double hh = ldexp(kp.rc, -c.en.z);
      const double ih = ldexp(kp.irc, c.en.z);
      v.w = hh * hh;
      w.x = (Real)sq[sidx];
      w.y = (Real)ih;
      w.z = (Real)(2.0 * ih * ih);
      set_slot_tg(w, tg);
      const double dx = v.x - cc[0], dy = v.y - cc[1], dz = v.z - cc[2];
      const double reach = hh + rho;
      live = !drop && fma(dx, dx, fma(dy, dy, dz * dz)) < reach * reach * (1.0 + 1e-12);
    } else {
      dead();
    }
  }
  __device__ void dead() {
    v.x = v.y = v.z = 1e30;
    v.w = 0;
    w.x = 0;
    w.y = 1;
    w.z = 2;
    set_slot_tg(w, -1);
    tg = -1;
    live = false;
  }
};

// Source ends of the pairs evaluated once: each pair's term q_t R goes to a
// row of RB slots x 64 lanes in LDS; after every RB slots of a tile, lane l
// adds the terms of slot l / LP from LP-th of the lanes (only the lanes whose
// targets meet that slot: lane % S == slot % S), LP lanes combine theirs, and
// one FP64 atomic per slot adds the sum to its target.
// FP64 rows padded to 68 entries (the flush's 16-byte reads of the RB rows
// fall on distinct banks); FP32 rows unpadded, so that the ring fits beside
// the staging slots at four waves per SIMD (its reads then share banks:
// measured faster than the padded ring at 3.75 waves).
template <class Real>
struct SymRing {
  static constexpr int RB = sizeof(Real) == 4 ? 16 : 8;   // slots per block
  static constexpr int LP = 64 / RB;                       // lanes per slot
  static constexpr int ROW = sizeof(Real) == 4 ? 64 : 68;
  static constexpr int SIZE = RB * ROW;
  __device__ static int at(int r, int col) { return r * ROW + col; }
};

// Data-parallel-primitive lane exchange (no LDS round trip): CTRL 0xB1 swaps
// neighbouring lanes (quad pattern 1,0,3,2), 0x4E lanes two apart (2,3,0,1),
// 0x141 mirrors each group of eight lanes.
template <int CTRL>
__device__ inline float dpp_x(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_x(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <class Real, int S>
__device__ inline void sym_flush(const Real* red, const typename SlotQ<Real>::T* shw, int slot0,
                                 double* __restrict__ pot, double cst) {
  using SR = SymRing<Real>;
  constexpr int PER = 64 / SR::LP;   // row entries per lane
  static_assert(PER % S == 0, "a lane's entries start at a multiple of S");
  static_assert(SR::LP == 4 || SR::LP == 8, "lanes of a slot: a quad or half a row");
  // the block is one wave and a wave's LDS operations complete in order: the
  // reads below see the block's writes; only the compiler must keep the order
  asm volatile("" ::: "memory");
  const int lane = threadIdx.x;
  const int j = lane / SR::LP, part = lane % SR::LP;
  const int tg = slot_tg(shw[slot0 + j]);   // read with the row entries
  Real sum = 0;
  if constexpr (S == 1) {
    Real s2 = 0;   // two chains of adds
#pragma unroll
    for (int i = 0; i < PER; i += 2) {
      sum += red[SR::at(j, part * PER + i)];
      s2 += red[SR::at(j, part * PER + i + 1)];
    }
    sum += s2;
  } else {
    const int i0 = j % S;
#pragma unroll
    for (int u = 0; u < PER / S; ++u) sum += red[SR::at(j, part * PER + i0 + u * S)];
  }
  sum += dpp_x<0xB1>(sum);
  sum += dpp_x<0x4E>(sum);
  if constexpr (SR::LP == 8) sum += dpp_x<0x141>(sum);
  if (part == 0 && tg >= 0) atomicAdd(&pot[tg], (double)sum * cst);
}

// One pass of a leaf's residual sums: 64 / S targets, S lanes per target,
// over the source list of the work item.  The lanes fetch 64 candidate
// sources at a time (the next round's loads in flight while a tile is
// summed); a candidate farther than h + rho from the centre cc of the pass's
// targets (all within rho of it) cannot reach any of them and is dropped,
// the others are appended to a ring of 128 LDS slots in lane order (ballot
// and prefix count).  Every 64 staged sources form a tile summed by all
// lanes; the last tile is padded with slots that never interact.  nlive
// counts the staged sources (the same on every lane).
// SYM: pairs evaluated once; qa is the lane's target charge, red the
// source-end ring (see sym_flush; the staged slots carry their targets).
template <int D, int NE, int S, bool GRAD, class Real, int NR, bool SYM>
__device__ void direct_pass(const KParams& kp, const int4* __restrict__ list, int lb, int le,
                            int pos0, int pos1, const double* __restrict__ sx,
                            const double* __restrict__ sq,
                            int64_t nimg, const double* cT, const double* x, const Real* ec,
                            const Real* edc, const double* cc, double rho, double4* shv,
                            typename SlotQ<Real>::T* shw, double& acc, double* g, int& nin,
                            int& nlive, const SymInfo& si, Real qa, Real* red,
                            double* __restrict__ pot, double cst) {
  const int lane = threadIdx.x;
  const int slice = lane % S;
  ListCursor cur;
  cur.init(list, lb, le, pos0 + lane, pos1);
  SourceSlot<Real> nxt;
  nxt.template fetch<SYM>(cur, kp, sx, sq, nimg, cT, D, cc, rho, si);
  // all lanes of the wave are active here, so the first active lane is lane 0
  bool more = __builtin_amdgcn_readfirstlane(cur.valid() ? 1 : 0) != 0;
  int head = 0, fill = 0;   // staged sources: ring slots [head, head + fill) mod 128
  while (more || fill > 0) {
    if (more) {
      const unsigned long long m = __builtin_amdgcn_ballot_w64(nxt.live);
      const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if (nxt.live) {
        const int sl = (head + fill + off) & 127;
        shv[sl] = nxt.v;
        shw[sl] = nxt.w;
      }
      const int nm = __builtin_amdgcn_readfirstlane((int)__popcll(m));
      fill += nm;
      nlive += nm;
      cur.advance(list);
      nxt.template fetch<SYM>(cur, kp, sx, sq, nimg, cT, D, cc, rho, si);
      more = __builtin_amdgcn_readfirstlane(cur.valid() ? 1 : 0) != 0;
      if (fill < 64 && more) continue;
    }
    const int base = head & 127;
    if (fill < 64 && lane >= fill) {
      // the last tile: slots past the staged sources never interact
      SourceSlot<Real> d;
      d.dead();
      shv[base + lane] = d.v;
      shw[base + lane] = d.w;
    }
    __syncthreads();
    Real ta = 0, tb = 0, ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
    const double4* tv = shv + base;
    const typename SlotQ<Real>::T* tw = shw + base;
    if constexpr (SYM) {
      // blocks of RB slots; the lane's slots of a block are u S + slice
      using SR = SymRing<Real>;
      constexpr int RB = SR::RB;
      static_assert(RB % S == 0, "a block holds whole rounds of the S lanes of a target");
#pragma unroll
      for (int b0 = 0; b0 < 64; b0 += RB) {
#pragma unroll
        for (int u = 0; u < RB / S; ++u) {
          const int r = u * S + slice;   // row in the block (static when S = 1)
          Real as;
          residual_pair<D, NE, false, Real, NR, true>(x, tv[b0 + r], tw[b0 + r], ec, edc,
                                                      (u & 1) ? tb : ta, ga, nin, qa, &as);
          red[SR::at(r, lane)] = as;
        }
        sym_flush<Real, S>(red, shw, base + b0, pot, cst);
        asm volatile("" ::: "memory");   // the block's reads precede the next writes
      }
    } else if constexpr (S == 1) {
      // one lane per target: the whole tile unrolled (LDS reads at immediate offsets)
#pragma unroll
      for (int k = 0; k < 64; k += 2) {
        residual_pair<D, NE, GRAD, Real, NR>(x, tv[k], tw[k], ec, edc, ta, ga, nin);
        residual_pair<D, NE, GRAD, Real, NR>(x, tv[k + 1], tw[k + 1], ec, edc, tb, gb, nin);
      }
    } else {
      // trip count independent of the lane (64 is a multiple of 2 S)
#pragma unroll 2
      for (int kk = 0; kk < 64; kk += 2 * S) {
        const int k = kk + slice;
        residual_pair<D, NE, GRAD, Real, NR>(x, tv[k], tw[k], ec, edc, ta, ga, nin);
        residual_pair<D, NE, GRAD, Real, NR>(x, tv[k + S], tw[k + S], ec, edc, tb, gb, nin);
      }
    }
    acc += (double)ta + (double)tb;
    if (GRAD)
      for (int a = 0; a < D; ++a) g[a] += (double)ga[a] + (double)gb[a];
    __syncthreads();   // the tile is read before its slots are staged again
    head += 64;
    fill = fill > 64 ? fill - 64 : 0;
  }
#pragma unroll
  for (int m = 1; m < S; m <<= 1) {
    acc += __shfl_xor(acc, m);
    if (GRAD)
      for (int a = 0; a < D; ++a) g[a] += __shfl_xor(g[a], m);
  }
}

// Leaf residual sums (the R part of the near field; interaction rule in
// k_leaf_lists).  One 64-lane block per work item = (target leaf, chunk of
// kDirectTgt targets, segment of kDirectSeg sources of its list), in
// decreasing order of cost.  The segments of a leaf add into the zeroed
// outputs with FP64 atomics; the first one also removes the self term.
// Positions are offsets from the target leaf's centre in FP64; Real = double:
// FP64 throughout; Real = float: the series, rsqrt and the sums over one tile
// of 64 sources in FP32, FP64 across tiles.
// SYM (targets = sources, no gradients, atomic mode; the lists skip the
// boxes whose pairs the later leaves evaluate): every pair of points in
// different leaves is evaluated once, its term q_s R added to the target and
// q_t R to the source's own target entry (itrg), oq holding the targets'
// charges in sorted order.
#define PDMK_DIRECT_PARAMS                                                                   \
    KParams kp, int nitems, const int2 *__restrict__ items, const int *__restrict__ lf_nsrc,    \
    const Level *__restrict__ lev, const int *__restrict__ lf_level,                            \
    const int *__restrict__ lf_box, const int *__restrict__ lbeg, const int4 *__restrict__ list, \
    const double *__restrict__ sx, const double *__restrict__ sq, int64_t nimg,                 \
    const double *__restrict__ tx, int64_t ntrg, const int *__restrict__ tperm,                 \
    const double *__restrict__ qorig, int self_targets, const double *__restrict__ Ec,          \
    const double *__restrict__ Edc, double *__restrict__ pot, double *__restrict__ grad,        \
    unsigned long long *__restrict__ n_support, double *__restrict__ part,                      \
    double *__restrict__ gpart, const int *__restrict__ item_beg, const int *__restrict__ itrg, \
    const double *__restrict__ oq
#define PDMK_DIRECT_ARGS                                                                      \
  kp, nitems, items, lf_nsrc, lev, lf_level, lf_box, lbeg, list, sx, sq, nimg, tx, ntrg, tperm, \
      qorig, self_targets, Ec, Edc, pot, grad, n_support, part, gpart, item_beg, itrg, oq
template <int D, int NE, bool GRAD, class Real, int NR, bool SYM>
__device__ __forceinline__ void direct_body(PDMK_DIRECT_PARAMS) {
  __shared__ double4 shv[128];
  __shared__ typename SlotQ<Real>::T shw[128];
  __shared__ Real red[SYM ? SymRing<Real>::SIZE : 1];
  if ((int)blockIdx.x >= nitems) return;
  const int2 item = items[blockIdx.x];
  const int i = item.x;
  const int nsrc = lf_nsrc[i];
  const int nseg = (nsrc + kDirectSeg - 1) / kDirectSeg;
  const int seg = item.y % nseg, tchunk = item.y / nseg;
  const int pos0 = seg * kDirectSeg;
  const int pos1 = min(nsrc, pos0 + kDirectSeg);
  // series coefficients (monomials in u, zero-padded to NE)
  Real ec[NE], edc[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    ec[k] = (Real)Ec[k];
    edc[k] = GRAD ? (Real)Edc[k] : (Real)0;
  }
  const int lane = threadIdx.x;
  const int lvl = lf_level[i], b = lf_box[i];
  const Level& T = lev[lvl];
  const int tb = T.tbeg[b] + tchunk * kDirectTgt;
  const int te = min(T.tend[b], tb + kDirectTgt);
  const int lb = lbeg[i], le = lbeg[i + 1];
  const double hT = kp.rc / (double)(1 << lvl);
  SymInfo si{itrg, 0, 0};
  if (SYM) {
    si.sb = T.sbeg[b];
    si.se = T.send[b];
  }
  const double cst = D == 3 ? kInv4Pi : kInv2Pi;
  double cT[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) cT[a] = kp.origin[a] + (T.coord[b * D + a] + 0.5) * hT;
  int nin = 0;
  long long nstaged = 0;   // staged sources x targets of the passes
  for (int t0 = tb; t0 < te;) {
    // lanes per target for this pass, from the targets still to do
    const int rem = te - t0;
    const int S = rem > 32 ? 1 : (rem > 16 ? 2 : (rem > 8 ? 4 : 8));
    const int t = t0 + lane / S;
    const bool valid = t < te;
    double x[3] = {0, 0, 0};
    // lanes of targets past the end sit far away: they stage sources but no
    // pair of theirs is inside the support
    for (int a = 0; a < D; ++a) x[a] = valid ? tx[a * ntrg + t] - cT[a] : 1e30;
    // bounding box of the pass's targets: centre cc, half-diagonal rho
    double cc[3] = {0, 0, 0}, rho2 = 0.0;
    for (int a = 0; a < D; ++a) {
      double lo = valid ? x[a] : 1e300, hi = valid ? x[a] : -1e300;
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, m));
        hi = fmax(hi, __shfl_xor(hi, m));
      }
      cc[a] = 0.5 * (lo + hi);
      rho2 += 0.25 * (hi - lo) * (hi - lo);
    }
    const double rho = sqrt(rho2);
    double acc = 0.0, g[3] = {0, 0, 0};
    int nin_p = 0, nlive = 0;
    const Real qa = (SYM && valid) ? (Real)oq[t] : (Real)0;
    switch (S) {
      case 1:
        direct_pass<D, NE, 1, GRAD, Real, NR, SYM>(kp, list, lb, le, pos0, pos1, sx, sq, nimg,
                                                   cT, x, ec, edc, cc, rho, shv, shw, acc, g,
                                                   nin_p, nlive, si, qa, red, pot, cst);
        break;
      case 2:
        direct_pass<D, NE, 2, GRAD, Real, NR, SYM>(kp, list, lb, le, pos0, pos1, sx, sq, nimg,
                                                   cT, x, ec, edc, cc, rho, shv, shw, acc, g,
                                                   nin_p, nlive, si, qa, red, pot, cst);
        break;
      case 4:
        direct_pass<D, NE, 4, GRAD, Real, NR, SYM>(kp, list, lb, le, pos0, pos1, sx, sq, nimg,
                                                   cT, x, ec, edc, cc, rho, shv, shw, acc, g,
                                                   nin_p, nlive, si, qa, red, pot, cst);
        break;
      default:
        direct_pass<D, NE, 8, GRAD, Real, NR, SYM>(kp, list, lb, le, pos0, pos1, sx, sq, nimg,
                                                   cT, x, ec, edc, cc, rho, shv, shw, acc, g,
                                                   nin_p, nlive, si, qa, red, pot, cst);
        break;
    }
    nin += nin_p;   // the same wave-wide count on every lane
    nstaged += (long long)nlive * ((te - t0 < 64 / S) ? te - t0 : 64 / S);
    if (valid && lane % S == 0) {
      double v = acc * cst;
      if (self_targets && seg == 0) {
        const double w0 = D == 3 ? kp.w0unit / hT : kp.w0unit - log(hT) * kInv2Pi;
        v -= qorig[tperm[t]] * w0;
      }
      if (part) {
        // fixed-order mode: this segment's partial sum, added by k_direct_reduce
        const int64_t slot = ((int64_t)item_beg[i] + item.y) * kDirectTgt + (t - tb);
        part[slot] = v;
        if (GRAD)
          for (int a = 0; a < D; ++a) gpart[slot * D + a] = g[a] * cst;
      } else {
        atomicAdd(&pot[t], v);
        if (GRAD)
          for (int a = 0; a < D; ++a) atomicAdd(&grad[(int64_t)t * D + a], g[a] * cst);
      }
    }
    t0 += 64 / S;
  }
  // pairs inside the support and staged pairs (statistics): one atomic pair
  // per block into one of kStatSlots slot pairs (one address for every block
  // serialises the atomics at the cache), folded by k_fold_stats
  if (lane == 0 && n_support) {
    unsigned long long* sl = n_support + 2 * (blockIdx.x & (kStatSlots - 1));
    atomicAdd(sl, (unsigned long long)nin);
    atomicAdd(sl + 1, (unsigned long long)nstaged);
  }
}

template <int D, int NE, bool GRAD, class Real, int NR, bool SYM>
__global__ __launch_bounds__(64) void k_direct(PDMK_DIRECT_PARAMS) {
  direct_body<D, NE, GRAD, Real, NR, SYM>(PDMK_DIRECT_ARGS);
}
// The FP32 pairs-once variant held to 128 registers (four waves per SIMD:
// measured faster than three without spills; FP64 is faster uncapped).
template <int D, int NE, bool GRAD, class Real, int NR, bool SYM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_direct_w4(
    PDMK_DIRECT_PARAMS) {
  direct_body<D, NE, GRAD, Real, NR, SYM>(PDMK_DIRECT_ARGS);
}

// Fixed-order completion of the residual sums: one block per work item in
// list order; the block of a chunk's first segment adds the chunk's segment
// partial sums in segment order (one thread per target, the only writer).
template <int D, bool GRAD>
__global__ __launch_bounds__(64) void k_direct_reduce(
    int nitems, const int2* __restrict__ items_u, const int* __restrict__ lf_nsrc,
    const Level* __restrict__ lev, const int* __restrict__ lf_level,
    const int* __restrict__ lf_box, const int* __restrict__ item_beg,
    const double* __restrict__ part, const double* __restrict__ gpart, double* __restrict__ pot,
    double* __restrict__ grad) {
  const int k = blockIdx.x;
  if (k >= nitems) return;
  const int2 it = items_u[k];
  const int i = it.x;
  const int nseg = (lf_nsrc[i] + kDirectSeg - 1) / kDirectSeg;
  if (it.y % nseg != 0) return;
  const int tchunk = it.y / nseg;
  const Level& T = lev[lf_level[i]];
  const int b = lf_box[i];
  const int tb = T.tbeg[b] + tchunk * kDirectTgt;
  const int te = min(T.tend[b], tb + kDirectTgt);
  const int t = tb + (int)threadIdx.x;
  if (t >= te) return;
  double v = 0.0, g[3] = {0.0, 0.0, 0.0};
  for (int sg = 0; sg < nseg; ++sg) {
    const int64_t slot =
        ((int64_t)item_beg[i] + tchunk * nseg + sg) * kDirectTgt + threadIdx.x;
    v += part[slot];
    if (GRAD)
      for (int a = 0; a < D; ++a) g[a] += gpart[slot * D + a];
  }
  pot[t] += v;
  if (GRAD)
    for (int a = 0; a < D; ++a) grad[(int64_t)t * D + a] += g[a];
}

// ------------------------------------------------------ source -> proxy charge
// Q_B[i0,i1,i2] = sum_s q_s l_i0(xi_0) l_i1(xi_1) l_i2(xi_2) over the sources of
// the childless children of the non-leaf box B, in B's scaled coordinates.
// A block owns one box; each thread owns one (i0, i1) pair (2D: one i0) and
// keeps the PMAX accumulators along the last axis in registers.  Lagrange rows
// of 32 sources at a time are staged in LDS.
template <int D, int PMAX, class Real>
__global__ __launch_bounds__(256) void k_anterp(KParams kp, Level L, Level C, int lvl,
                                                const double* __restrict__ sx,
                                                const double* __restrict__ sq, int64_t nimg,
                                                const double* __restrict__ nodes,
                                                const double* __restrict__ bw,
                                                Real* __restrict__ Q) {
  constexpr int TS = 32;
  __shared__ Real rows[TS * D * PMAX];
  __shared__ Real qs[TS];
  const int p = kp.p;
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  const int pD = D == 3 ? p * p * p : p * p;
  const int npair = D == 3 ? p * p : p;
  const double h = kp.rc / (double)(1 << lvl);
  double cen[D];
  for (int a = 0; a < D; ++a) cen[a] = kp.origin[a] + (L.coord[b * D + a] + 0.5) * h;
  const double sc = 2.0 / h;
  const int c0 = L.child0[b];
  for (int pr0 = 0; pr0 < npair; pr0 += 256) {
    const int pr = pr0 + threadIdx.x;
    const bool act = pr < npair;
    const int i0 = D == 3 ? (act ? pr / p : 0) : (act ? pr : 0);
    const int i1 = D == 3 ? (act ? pr % p : 0) : 0;
    Real acc[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) acc[j] = 0;
    for (int o = 0; o < (1 << D); ++o) {
      const int c = c0 + o;
      if (C.child0[c] >= 0) continue;   // non-leaf child: handled by the transfer
      const int sb = C.sbeg[c], se = C.send[c];
      for (int s0 = sb; s0 < se; s0 += TS) {
        const int ns = min(TS, se - s0);
        __syncthreads();
        if (threadIdx.x < ns * D) {
          const int si = threadIdx.x / D, a = threadIdx.x % D;
          const double xi = (sx[a * nimg + s0 + si] - cen[a]) * sc;
          lagrange_rows<Real>(p, nodes, bw, xi, rows + (si * D + a) * PMAX, (Real*)nullptr);
        }
        if (threadIdx.x < ns) qs[threadIdx.x] = (Real)sq[s0 + threadIdx.x];
        __syncthreads();
        for (int si = 0; si < ns; ++si) {
          const Real* rw = rows + si * D * PMAX;
          Real wv = qs[si] * rw[i0];
          if (D == 3) wv *= rw[PMAX + i1];
          const Real* rl = rw + (D - 1) * PMAX;
#pragma unroll
          for (int j = 0; j < PMAX; ++j) acc[j] = fma(wv, rl[j], acc[j]);
        }
      }
    }
    if (act) {
      Real* out = Q + (int64_t)k * pD + (int64_t)pr * p;
#pragma unroll
      for (int j = 0; j < PMAX; ++j)
        if (j < p) out[j] = acc[j];
    }
  }
}

// ------------------------------------------- tensor-product child <-> parent
// Transfer of proxy data between a non-leaf child (level l+1, index kc among
// non-leaf boxes) and its parent (level l):
//   up   : out[P] = sum_i T_sigma[P][i] in[i]    (charges, child -> parent)
//   down : out[i] = sum_P T_sigma[P][i] in[P]    (potentials, parent -> child)
// applied along every axis.  One block per child: the tensor sits in LDS and
// each thread transforms whole 1D lines in place (a line is read into
// registers before it is overwritten).  Up adds into the parent with atomics
// (siblings share it), down adds into the child.
// In-place 1D transforms of all lines of the tensor along each axis.  tm
// holds, per octant bit, the matrix column-wise and zero-padded to PMAX:
// tm[sel][i][o] is the weight of input i for output o.  Each thread keeps the
// PMAX outputs of its line in independent accumulators.
template <int D, int PMAX, bool LDS, class Real>
__device__ inline void transfer_lines(int p, int pD, int oct, Real* ten, const Real* tm) {
  const int nlines = pD / p;
  for (int ax = 0; ax < D; ++ax) {
    const Real* M = tm + ((oct >> ax) & 1) * p * PMAX;
    const int stride = D == 3 ? (ax == 0 ? p * p : (ax == 1 ? p : 1)) : (ax == 0 ? p : 1);
    for (int ln = threadIdx.x; ln < nlines; ln += blockDim.x) {
      int base;
      if (D == 3) {
        const int u = ln / p, v = ln % p;
        base = ax == 0 ? u * p + v : (ax == 1 ? u * p * p + v : u * p * p + v * p);
      } else {
        base = ax == 0 ? ln : ln * p;
      }
      Real acc[PMAX];
#pragma unroll
      for (int o = 0; o < PMAX; ++o) acc[o] = 0;
      for (int i = 0; i < p; ++i) {
        const Real vi = ten[base + i * stride];
        const Real* col = M + i * PMAX;
#pragma unroll
        for (int o = 0; o < PMAX; ++o) acc[o] = fma(col[o], vi, acc[o]);
      }
#pragma unroll
      for (int o = 0; o < PMAX; ++o)
        if (o < p) ten[base + o * stride] = acc[o];
    }
    __syncthreads();
  }
}

// MODE 0: up, one block per parent (register accumulation, NOWN entries per
// thread); MODE 1: up, one block per child with atomic adds into the parent
// (large tensors); MODE 2: down, one block per child.
template <int D, int PMAX, bool LDS, int NOWN, int MODE, class Real>
__global__ __launch_bounds__(256) void k_transfer(KParams kp, Level Lp, Level Lc,
                                                  const Real* __restrict__ src,
                                                  Real* __restrict__ dst,
                                                  const double* __restrict__ Tm,
                                                  Real* __restrict__ scratch, int oct_only) {
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* sm = reinterpret_cast<Real*>(smraw);
  const int p = kp.p;
  const int pD = D == 3 ? p * p * p : p * p;
  const int blk = blockIdx.x;
  // the tensor lives in LDS when it fits, else in this block's global scratch
  Real* ten = LDS ? sm : scratch + (int64_t)blk * pD;
  Real* tm = LDS ? sm + pD : sm;  // 2 p PMAX
  // Tm[sel][P][i] = l_P(child node i).  Up maps input i -> output P, down maps
  // input P -> output i.
  for (int e = threadIdx.x; e < 2 * p * PMAX; e += blockDim.x) {
    const int sel = e / (p * PMAX), r = (e / PMAX) % p, o = e % PMAX;
    double v = 0.0;
    if (o < p) v = MODE == 2 ? Tm[sel * p * p + r * p + o] : Tm[sel * p * p + o * p + r];
    tm[e] = (Real)v;
  }
  __syncthreads();
  if (MODE == 0) {
    const int P = Lp.nl_box[blk];
    const int c0 = Lp.child0[P];
    Real acc[NOWN];
#pragma unroll
    for (int r = 0; r < NOWN; ++r) acc[r] = 0;
    bool any = false;
    for (int o = 0; o < (1 << D); ++o) {
      const int kc = Lc.nlid[c0 + o];
      if (kc < 0) continue;
      any = true;
      const Real* in = src + (int64_t)kc * pD;
      __syncthreads();
      for (int e = threadIdx.x; e < pD; e += blockDim.x) ten[e] = in[e];
      __syncthreads();
      transfer_lines<D, PMAX, LDS, Real>(p, pD, o, ten, tm);
#pragma unroll
      for (int r = 0; r < NOWN; ++r) {
        const int e = threadIdx.x + r * 256;
        if (e < pD) acc[r] += ten[e];
      }
    }
    if (!any) return;
    Real* out = dst + (int64_t)blk * pD;
#pragma unroll
    for (int r = 0; r < NOWN; ++r) {
      const int e = threadIdx.x + r * 256;
      if (e < pD) out[e] += acc[r];
    }
  } else {
    const int kc = blk;
    const int c = Lc.nl_box[kc];
    const int pb = Lc.parent[c];
    const int kpar = Lp.nlid[pb];
    const int oct = c - Lp.child0[pb];
    // fixed-order mode: one octant per launch, so a parent receives one add
    if (oct_only >= 0 && oct != oct_only) return;
    const Real* in = src + (int64_t)(MODE == 1 ? kc : kpar) * pD;
    for (int e = threadIdx.x; e < pD; e += blockDim.x) ten[e] = in[e];
    __syncthreads();
    transfer_lines<D, PMAX, LDS, Real>(p, pD, oct, ten, tm);
    if (MODE == 1) {
      Real* out = dst + (int64_t)kpar * pD;
      for (int e = threadIdx.x; e < pD; e += blockDim.x) atomicAdd(out + e, ten[e]);
    } else {
      Real* out = dst + (int64_t)kc * pD;
      for (int e = threadIdx.x; e < pD; e += blockDim.x) out[e] += ten[e];
    }
  }
}

// --------------------------------------------------- plane-wave transforms
// Contract one axis of a batch of tensors with a complex matrix.
// in : [nitems][n0][n1][n2] (real or complex), out: same with dim[ax] = mout.
// Coefficient for output index o and contracted index i:
//   trans = 0: M[(row0 + o) * ld + i]     trans = 1: M[(row0 + i) * ld + o]
// optionally conjugated.  MODE 0 stores complex; MODE 1 adds the weighted real
// part to a real output (weight 1 for contracted index 0, 2 otherwise: the
// Hermitian half of the first axis).
template <bool IN_CPLX, int MODE>
__global__ void k_axis(int nitems, int n0, int n1, int n2, int ax, int mout,
                       const void* __restrict__ in_, void* __restrict__ out_,
                       const double2* __restrict__ M, int row0, int ld, int trans, int conj) {
  int dims[3] = {n0, n1, n2};
  int od[3] = {n0, n1, n2};
  od[ax] = mout;
  const int64_t osz = (int64_t)od[0] * od[1] * od[2];
  const int64_t isz = (int64_t)n0 * n1 * n2;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= osz * nitems) return;
  const int64_t item = gid / osz;
  const int64_t e = gid % osz;
  int o[3];
  o[2] = (int)(e % od[2]);
  o[1] = (int)((e / od[2]) % od[1]);
  o[0] = (int)(e / ((int64_t)od[2] * od[1]));
  int istr[3] = {n1 * n2, n2, 1};
  int64_t ibase = item * isz;
  for (int a = 0; a < 3; ++a)
    if (a != ax) ibase += (int64_t)o[a] * istr[a];
  const int oi = o[ax];
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < dims[ax]; ++i) {
    double2 m = trans ? M[(row0 + i) * ld + oi] : M[(row0 + oi) * ld + i];
    if (conj) m.y = -m.y;
    if (IN_CPLX) {
      const double2 v = reinterpret_cast<const double2*>(in_)[ibase + (int64_t)i * istr[ax]];
      if (MODE == 1) {
        const double w = i == 0 ? 1.0 : 2.0;
        sr += w * (m.x * v.x - m.y * v.y);
      } else {
        sr += m.x * v.x - m.y * v.y;
        si += m.x * v.y + m.y * v.x;
      }
    } else {
      const double v = reinterpret_cast<const double*>(in_)[ibase + (int64_t)i * istr[ax]];
      sr += m.x * v;
      si += m.y * v;
    }
  }
  if (MODE == 1) reinterpret_cast<double*>(out_)[gid] += sr;
  else reinterpret_cast<double2*>(out_)[gid] = make_double2(sr, si);
}

// The same contraction as k_axis (complex input and output, MODE 0) as one
// library GEMM on the matrix cores: with the tensor [nitems][n0][n1][n2] split
// at the contracted axis into (outer, n_i, inner), the output is
//   out[b][o][r] = sum_i Mc(o, i) in[b][i][r],   Mc(o, i) = M[(row0 + o) ld + i]
// (trans = 0) or M[(row0 + i) ld + o] (trans = 1).  Column-major views: for
// inner > 1 a strided batch over b of C (inner x mout) = X (inner x n_i)
// op(B); for inner = 1 one product C (mout x rows) = op(A) X (n_i x rows).
// Conjugation comes from the conjugated tables (trans = 0) or the conjugate
// transpose (trans = 1).
static void axis_gemm(pdmk_plan* P, hipStream_t s, int nitems, int n0, int n1, int n2, int ax,
                      int mout, const double2* in, double2* out, const double2* M,
                      const double2* Mconj, int row0, int ld, int trans, int conj) {
  rocblas_handle h = static_cast<rocblas_handle>(P->blas);
  if (!h) {
    if (rocblas_create_handle(&h) != rocblas_status_success)
      throw Error{PDMK_ERR_HIP, "rocblas_create_handle failed"};
    P->blas = h;
  }
  if (rocblas_set_stream(h, s) != rocblas_status_success)
    throw Error{PDMK_ERR_HIP, "rocblas_set_stream failed"};
  const int dims[3] = {n0, n1, n2};
  const int ni = dims[ax];
  int64_t outer = nitems, inner = 1;
  for (int a = 0; a < ax; ++a) outer *= dims[a];
  for (int a = ax + 1; a < 3; ++a) inner *= dims[a];
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  auto cz = [](const double2* p) { return reinterpret_cast<const rocblas_double_complex*>(p); };
  rocblas_status st;
  if (inner == 1) {
    // C (mout x rows) = op(A) X; A from the table: trans = 0 -> A^T stored
    // (lda = ld), trans = 1 -> A stored (lda = ld, conj: the conjugated table)
    const int64_t rows = outer;
    if (rows > INT32_MAX) throw Error{PDMK_ERR_UNSUPPORTED, "GEMM rows beyond int32"};
    const double2* A = (trans ? (conj ? Mconj : M) : (conj ? Mconj : M)) + (int64_t)row0 * ld;
    const rocblas_operation opA = trans ? rocblas_operation_none : rocblas_operation_transpose;
    st = rocblas_zgemm(h, opA, rocblas_operation_none, mout, (int)rows, ni, &one, cz(A), ld,
                       cz(in), ni, &zero, reinterpret_cast<rocblas_double_complex*>(out), mout);
  } else {
    // per b: C (inner x mout) = X (inner x n_i) B, B(i, o) = Mc(o, i):
    // trans = 0 -> B stored (ldb = ld, conj: the conjugated table),
    // trans = 1 -> B^T stored (ldb = ld; conj: conjugate transpose)
    if (outer > INT32_MAX || inner > INT32_MAX) throw Error{PDMK_ERR_UNSUPPORTED, "GEMM shape"};
    const double2* B = (trans ? M : (conj ? Mconj : M)) + (int64_t)row0 * ld;
    const rocblas_operation opB = trans ? (conj ? rocblas_operation_conjugate_transpose
                                                : rocblas_operation_transpose)
                                        : rocblas_operation_none;
    st = rocblas_zgemm_strided_batched(h, rocblas_operation_none, opB, (int)inner, mout, ni, &one,
                                       cz(in), (int)inner, (rocblas_stride)(ni * inner), cz(B), ld,
                                       0, &zero, reinterpret_cast<rocblas_double_complex*>(out),
                                       (int)inner, (rocblas_stride)(mout * inner), (int)outer);
  }
  if (st != rocblas_status_success)
    throw Error{PDMK_ERR_HIP, "rocblas_zgemm failed: " + std::string(rocblas_status_to_string(st))};
}

void gemm_release(pdmk_plan* P) {
  if (P->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(P->blas));
  P->blas = nullptr;
}

// real -> complex (im = 0)
__global__ void k_real_to_cplx(int64_t n, const double* __restrict__ in, double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2(in[i], 0.0);
}
// Full (J+1) x n x n mode grid <-> compact half-ball order of a chunk of
// boxes: gather S[k][e] = full[k][mode(e)]; scatter writes every full mode
// (zero outside the ball, and for boxes without targets, whose incoming
// expansions the translation leaves unwritten).
__global__ void k_gather_ball(int nc, int nball, int J, const int* __restrict__ ball,
                              const double2* __restrict__ full, double2* __restrict__ S) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nc * nball) return;
  const int k = (int)(gid / nball), e = (int)(gid - (int64_t)k * nball);
  const int n = 2 * J + 1;
  const int c = ball[e];
  const int j0 = c & 255, a = (c >> 8) & 255, b = c >> 16;
  S[gid] = full[(int64_t)k * (J + 1) * n * n + ((int64_t)j0 * n + a) * n + b];
}
__global__ void k_scatter_ball(int nc, int k0, Level L, int nball, int J,
                               const int2* __restrict__ brow, const double2* __restrict__ Iw,
                               double2* __restrict__ full) {
  const int n = 2 * J + 1;
  const int64_t msz = (int64_t)(J + 1) * n * n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nc * msz) return;
  const int k = (int)(gid / msz);
  const int64_t m = gid - (int64_t)k * msz;
  const int r = (int)(m / n), b = (int)(m - (int64_t)r * n);
  const int bx = L.nl_box[k0 + k];
  double2 v = make_double2(0.0, 0.0);
  if (L.tend[bx] > L.tbeg[bx]) {
    const int2 rw = brow[r];   // {compact index of j2 = -J, half width}
    if (rw.y >= 0 && b - J >= -rw.y && b - J <= rw.y)
      v = Iw[(int64_t)(k0 + k) * nball + rw.x + b];
  }
  full[gid] = v;
}

// out += Re(in)
__global__ void k_add_real(int64_t n, const double2* __restrict__ in, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += in[i].x;
}

// Incoming expansion of every non-leaf box B of a level:
//   I_B(j) = c_l(|j|^2) sum_{C} omega^{j.(c_B - c_C)/h} S_C(j),
// over the non-leaf colleagues C (including B), omega = exp(2 pi i / 3).
template <int D>
__global__ void k_translate(Level L, int J, int k0, int nk, const double2* __restrict__ S,
                            double2* __restrict__ I, const double* __restrict__ dtab,
                            double levfac, unsigned long long* __restrict__ npairs) {
  const int n1 = 2 * J + 1;
  const int msz = D == 3 ? (J + 1) * n1 * n1 : (J + 1) * n1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)msz * nk) return;
  const int k = k0 + (int)(gid / msz), m = (int)(gid % msz);
  int j[3] = {0, 0, 0};
  if (D == 3) {
    j[2] = m % n1 - J;
    j[1] = (m / n1) % n1 - J;
    j[0] = m / (n1 * n1);
  } else {
    j[1] = m % n1 - J;
    j[0] = m / n1;
  }
  const int b = L.nl_box[k];
  const int ncoll = D == 3 ? 27 : 9;
  const double2 w3[3] = {make_double2(1.0, 0.0), make_double2(-0.5, 0.8660254037844386),
                         make_double2(-0.5, -0.8660254037844386)};
  double sr = 0.0, si = 0.0;
  int cnt = 0;
  for (int sl = 0; sl < ncoll; ++sl) {
    const int c = L.coll[b * ncoll + sl];
    if (c < 0) continue;
    const int kc = L.nlid[c];
    if (kc < 0) continue;
    ++cnt;
    // slot encodes coord(C) - coord(B) + 1 per axis; delta = coord(B) - coord(C)
    int ph = 0, t = sl;
    for (int a = 0; a < D; ++a) {
      const int dl = t % 3 - 1;
      t /= 3;
      ph -= j[a] * dl;
    }
    ph %= 3;
    if (ph < 0) ph += 3;
    const double2 v = S[(int64_t)kc * msz + m];
    const double2 w = w3[ph];
    sr += w.x * v.x - w.y * v.y;
    si += w.x * v.y + w.y * v.x;
  }
  const int nn = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
  const double cf = levfac * dtab[nn];
  I[gid] = make_double2(cf * sr, cf * si);
  if (m == 0 && npairs) atomicAdd(npairs, (unsigned long long)cnt);
}

// ------------------------------------------- fused per-box plane waves (3D)
// Outgoing expansion of a non-leaf box, one slab j0 (Hermitian half, j0 >= 0)
// at a time:  x = F_a Q (contract the first axis), z = F_b x, S[j0] = z F_c^T,
// with F[j][i] = exp(-i pi j xi_i / 3).  The proxy tensor and the small
// factors sit in LDS; S goes to global memory.
template <class R> struct CplxOf;
template <> struct CplxOf<double> { using T = double2; };
template <> struct CplxOf<float> { using T = float2; };
template <class R> using Cx = typename CplxOf<R>::T;

template <class C>
__device__ inline C cfma(C a, C b, C c) {   // a * b + c
  C r;
  r.x = fma(a.x, b.x, fma(-a.y, b.y, c.x));
  r.y = fma(a.x, b.y, fma(a.y, b.x, c.y));
  return r;
}
template <class C>
__device__ inline C cfma_conj_a(C a, C b, C c) {   // conj(a) * b + c
  C r;
  r.x = fma(a.x, b.x, fma(a.y, b.y, c.x));
  r.y = fma(a.x, b.y, fma(-a.y, b.x, c.y));
  return r;
}

template <class Real>
__global__ __launch_bounds__(256) void k_pw_out(KParams kp, Level L, const Real* __restrict__ Q,
                                                const Cx<Real>* __restrict__ F,
                                                Cx<Real>* __restrict__ S) {
  using C = Cx<Real>;
  extern __shared__ __align__(16) unsigned char smraw[];
  const int p = kp.p, J = kp.J, n = 2 * J + 1;
  const int p2 = p * p, p3 = p2 * p;
  C* f = reinterpret_cast<C*>(smraw);                 // n x p
  C* fT = f + n * p;                                  // p x n
  C* x = fT + n * p;                                  // p x p
  C* z = x + p2;                                      // n x p
  Real* q = reinterpret_cast<Real*>(z + n * p);       // p^3
  const int k = blockIdx.x;
  const Real* Qk = Q + (int64_t)k * p3;
  for (int e = threadIdx.x; e < p3; e += 256) q[e] = Qk[e];
  for (int e = threadIdx.x; e < n * p; e += 256) {
    const C v = F[e];
    f[e] = v;
    fT[(e % p) * n + e / p] = v;
  }
  __syncthreads();
  const int msz = (J + 1) * n * n;
  const C zero = {0, 0};
  for (int j0 = 0; j0 <= J; ++j0) {
    const C* fr = f + (J + j0) * p;
    for (int e = threadIdx.x; e < p2; e += 256) {
      C acc = zero;
      for (int a = 0; a < p; ++a) {
        const Real v = q[a * p2 + e];
        acc.x = fma(fr[a].x, v, acc.x);
        acc.y = fma(fr[a].y, v, acc.y);
      }
      x[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * p; e += 256) {
      const int j1 = e / p, c = e % p;
      C acc = zero;
      for (int b = 0; b < p; ++b) acc = cfma(f[j1 * p + b], x[b * p + c], acc);
      z[e] = acc;
    }
    __syncthreads();
    C* Sk = S + (int64_t)k * msz + (int64_t)j0 * n * n;
    for (int e = threadIdx.x; e < n * n; e += 256) {
      const int j1 = e / n, j2 = e % n;
      C acc = zero;
      for (int c = 0; c < p; ++c) acc = cfma(z[j1 * p + c], fT[c * n + j2], acc);
      Sk[e] = acc;
    }
    __syncthreads();
  }
}

// Incoming expansion of a non-leaf box B holding targets, slab by slab:
//   I[j0] = c_l(|j|^2) sum_C omega^{j.(c_B - c_C)/h} S_C[j0]   (|j| <= J only)
// then plane waves -> proxy potential: z = I F_c^*, x = F_b^* z,
// phi += w(j0) Re(F_a^* x) with w = 1 for j0 = 0 and 2 otherwise.
template <class Real>
__global__ __launch_bounds__(256) void k_pw_in(KParams kp, Level L, const Cx<Real>* __restrict__ S,
                                               const Cx<Real>* __restrict__ F,
                                               const double* __restrict__ dtab, double levfac,
                                               Real* __restrict__ Phi,
                                               unsigned long long* __restrict__ npairs) {
  using C = Cx<Real>;
  extern __shared__ __align__(16) unsigned char smraw[];
  __shared__ int ckc[27], cph[27][3];
  __shared__ int ncol;
  const int p = kp.p, J = kp.J, n = 2 * J + 1;
  const int p2 = p * p, p3 = p2 * p;
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  if (L.tend[b] <= L.tbeg[b]) return;   // no targets below this box
  C* f = reinterpret_cast<C*>(smraw);                 // n x p
  C* slab = f + n * p;                                // n x n
  C* z = slab + n * n;                                // n x p
  C* x = z + n * p;                                   // p x p
  Real* phi = reinterpret_cast<Real*>(x + p2);        // p^3
  if (threadIdx.x == 0) {
    int m = 0;
    for (int sl = 0; sl < 27; ++sl) {
      const int c = L.coll[b * 27 + sl];
      if (c < 0 || L.nlid[c] < 0) continue;
      ckc[m] = L.nlid[c];
      cph[m][0] = -(sl % 3 - 1);
      cph[m][1] = -((sl / 3) % 3 - 1);
      cph[m][2] = -(sl / 9 - 1);
      ++m;
    }
    ncol = m;
    if (npairs) {
      atomicAdd(npairs, (unsigned long long)m);
      atomicAdd(npairs + 1, 1ull);
    }
  }
  for (int e = threadIdx.x; e < p3; e += 256) phi[e] = 0;
  for (int e = threadIdx.x; e < n * p; e += 256) f[e] = F[e];
  __syncthreads();
  const int nc = ncol;
  const int msz = (J + 1) * n * n;
  const C zero = {0, 0};
  const C w3[3] = {{(Real)1, (Real)0}, {(Real)-0.5, (Real)0.8660254037844386},
                   {(Real)-0.5, (Real)-0.8660254037844386}};
  for (int j0 = 0; j0 <= J; ++j0) {
    for (int e = threadIdx.x; e < n * n; e += 256) {
      const int j1 = e / n - J, j2 = e % n - J;
      const int nn = j0 * j0 + j1 * j1 + j2 * j2;
      C acc = zero;
      if (nn <= J * J) {
        for (int m = 0; m < nc; ++m) {
          int ph = (j0 * cph[m][0] + j1 * cph[m][1] + j2 * cph[m][2]) % 3;
          if (ph < 0) ph += 3;
          const C v = S[(int64_t)ckc[m] * msz + (int64_t)j0 * n * n + e];
          acc = cfma(w3[ph], v, acc);
        }
        const Real cf = (Real)(levfac * dtab[nn]);
        acc.x *= cf;
        acc.y *= cf;
      }
      slab[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * p; e += 256) {
      const int j1 = e / p, c = e % p;
      C acc = zero;
      for (int j2 = 0; j2 < n; ++j2) acc = cfma_conj_a(f[j2 * p + c], slab[j1 * n + j2], acc);
      z[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < p2; e += 256) {
      const int bb = e / p, c = e % p;
      C acc = zero;
      for (int j1 = 0; j1 < n; ++j1) acc = cfma_conj_a(f[j1 * p + bb], z[j1 * p + c], acc);
      x[e] = acc;
    }
    __syncthreads();
    const Real w = j0 == 0 ? (Real)1 : (Real)2;
    const C* fr = f + (J + j0) * p;
    for (int e = threadIdx.x; e < p3; e += 256) {
      const int a = e / p2, bc = e % p2;
      const C fa = fr[a], xv = x[bc];
      phi[e] = fma(w, fa.x * xv.x + fa.y * xv.y, phi[e]);   // Re(conj(fa) xv)
    }
    __syncthreads();
  }
  Real* out = Phi + (int64_t)k * p3;
  for (int e = threadIdx.x; e < p3; e += 256) out[e] += phi[e];
}

// -------------------------------------------------- proxy potential -> targets
// Targets of the childless children of a non-leaf box P evaluate P's proxy
// potential (one block per P, one thread per target).  The potential tensor is
// read through the scalar cache (uniform addresses); the Lagrange rows of the
// last axis live in registers, the others in LDS (transposed, conflict free).
template <class Real>
using const_rptr = const Real __attribute__((address_space(4)))*;

template <int D, int PMAX, int NT, bool GRAD, class Real>
__global__ __launch_bounds__(NT) void k_eval_children(
    KParams kp, Level Lp, Level Lc, int lvl, const double* __restrict__ tx, int64_t ntrg,
    const double* __restrict__ nodes, const double* __restrict__ bw,
    double* __restrict__ pot, double* __restrict__ grad) {
  constexpr int NR = GRAD ? 2 : 1;
  __shared__ Real lrow[NR * (D - 1) * PMAX * NT];   // rows (and derivative rows) of axes < D-1
  __shared__ int cb[8], cpre[9];
  const int p = kp.p;
  const int k = blockIdx.x;
  const int P = Lp.nl_box[k];
  const int c0 = Lp.child0[P];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int o = 0; o < (1 << D); ++o) {
      const int c = c0 + o;
      cpre[o] = acc;
      if (Lc.child0[c] < 0) {
        cb[o] = Lc.tbeg[c];
        acc += Lc.tend[c] - Lc.tbeg[c];
      } else {
        cb[o] = 0;
      }
    }
    cpre[1 << D] = acc;
  }
  __syncthreads();
  const int total = cpre[1 << D];
  if (total == 0) return;
  const int pD = D == 3 ? p * p * p : p * p;
  const_rptr<Real> Phi = (const_rptr<Real>)((const Real*)Lp.proxy_phi + (int64_t)k * pD);
  const double hP = kp.rc / (double)(1 << lvl);
  double cen[D];
  for (int a = 0; a < D; ++a) cen[a] = kp.origin[a] + (Lp.coord[P * D + a] + 0.5) * hP;
  const double sc = 2.0 / hP;
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < total; j0 += NT) {
    const int j = j0 + tid;
    const bool valid = j < total;
    int t = 0;
    if (valid) {
      int o = 0;
      while (o + 1 < (1 << D) && cpre[o + 1] <= j) ++o;
      t = cb[o] + (j - cpre[o]);
    }
    double rld[PMAX], dld[PMAX];
    Real rl[PMAX], dl[PMAX];
    for (int a = 0; a < D; ++a) {
      const double xi = valid ? (tx[a * ntrg + t] - cen[a]) * sc : 0.0;
      lagrange_rows_reg<PMAX, GRAD>(p, nodes, bw, xi, rld, dld);
#pragma unroll
      for (int m = 0; m < PMAX; ++m) {
        rl[m] = (Real)rld[m];
        dl[m] = GRAD ? (Real)dld[m] : (Real)0;
      }
      if (a < D - 1) {
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
          lrow[(a * PMAX + m) * NT + tid] = rl[m];
          if (GRAD) lrow[(((D - 1) + a) * PMAX + m) * NT + tid] = dl[m];
        }
      }
    }
    // rl / dl now hold the last axis
    Real acc = 0, g0 = 0, g1 = 0, g2 = 0;
    if (D == 3) {
      for (int i0 = 0; i0 < p; ++i0) {
        Real a1 = 0, a1g1 = 0, a1g2 = 0;
        for (int i1 = 0; i1 < p; ++i1) {
          const_rptr<Real> ph = Phi + (i0 * p + i1) * p;
          // PMAX consecutive values (entries past p meet zero rows; the
          // buffer carries PMAX zeros of padding at its end)
          Real v[PMAX];
#pragma unroll
          for (int m = 0; m < PMAX; ++m) v[m] = ph[m];
          Real a2 = 0, a2d = 0;
#pragma unroll
          for (int m = 0; m < PMAX; ++m) {
            a2 = fma(v[m], rl[m], a2);
            if (GRAD) a2d = fma(v[m], dl[m], a2d);
          }
          const Real r1 = lrow[(PMAX + i1) * NT + tid];
          a1 = fma(r1, a2, a1);
          if (GRAD) {
            a1g1 = fma(lrow[(((D - 1) + 1) * PMAX + i1) * NT + tid], a2, a1g1);
            a1g2 = fma(r1, a2d, a1g2);
          }
        }
        const Real r0 = lrow[i0 * NT + tid];
        acc = fma(r0, a1, acc);
        if (GRAD) {
          g0 = fma(lrow[((D - 1) * PMAX + i0) * NT + tid], a1, g0);
          g1 = fma(r0, a1g1, g1);
          g2 = fma(r0, a1g2, g2);
        }
      }
    } else {
      for (int i0 = 0; i0 < p; ++i0) {
        const_rptr<Real> ph = Phi + i0 * p;
        Real v[PMAX];
#pragma unroll
        for (int m = 0; m < PMAX; ++m) v[m] = ph[m];
        Real a1 = 0, a1d = 0;
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
          a1 = fma(v[m], rl[m], a1);
          if (GRAD) a1d = fma(v[m], dl[m], a1d);
        }
        const Real r0 = lrow[i0 * NT + tid];
        acc = fma(r0, a1, acc);
        if (GRAD) {
          g0 = fma(lrow[((D - 1) * PMAX + i0) * NT + tid], a1, g0);
          g1 = fma(r0, a1d, g1);
        }
      }
    }
    if (valid) {
      pot[t] += (double)acc;
      if (GRAD) {
        grad[(int64_t)t * D + 0] += (double)g0 * sc;
        grad[(int64_t)t * D + 1] += (double)g1 * sc;
        if (D == 3) grad[(int64_t)t * D + 2] += (double)g2 * sc;
      }
    }
  }
}

template <int D, int NE, class Real>
static void launch_direct_t(const KParams& kp, Eval& E, pdmk_plan* P, hipStream_t s,
                            bool want_grad, unsigned long long* nsup) {
  const int off = sizeof(Real) == 4 ? 32 : 0;   // FP32 evaluation: the cut series
  const double* c = (D == 3 ? P->d_E : P->d_F2) + off;
  const double* cd = (D == 3 ? P->d_Ed : P->d_F2d) + off;
  // fixed-order mode: per-segment partial sums, then k_direct_reduce
  double* part = nullptr;
  double* gpart = nullptr;
  if (E.det) {
    part = E.alloc<double>((size_t)E.nitems * kDirectTgt);
    if (want_grad) gpart = E.alloc<double>((size_t)E.nitems * kDirectTgt * D);
  }
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(E.nitems), dim3(64), 0, s, kp, E.nitems, E.items, E.lf_nsrc,
                       E.d_lev, E.lf_level, E.lf_box, E.lf_list_beg, E.list, E.sx, E.sq, E.n_img,
                       E.tx, E.n_trg, E.tperm, E.q, E.self_targets ? 1 : 0, c, cd, E.pot_sorted,
                       E.grad_sorted, nsup, part, gpart, E.item_beg, E.img_trg, E.oq);
    if (E.det) {
      if (want_grad)
        hipLaunchKernelGGL((k_direct_reduce<D, true>), dim3(E.nitems), dim3(64), 0, s,
                           E.nitems, E.items_u, E.lf_nsrc, E.d_lev, E.lf_level, E.lf_box,
                           E.item_beg, part, gpart, E.pot_sorted, E.grad_sorted);
      else
        hipLaunchKernelGGL((k_direct_reduce<D, false>), dim3(E.nitems), dim3(64), 0, s,
                           E.nitems, E.items_u, E.lf_nsrc, E.d_lev, E.lf_level, E.lf_box,
                           E.item_beg, part, gpart, E.pot_sorted, E.grad_sorted);
    }
  };
  // FP64 3D: one Newton step of the reciprocal square root where eps >= 1e-10
  // (its error, below 1e-14, is then far under the tolerance), two below
  // pairs evaluated once: only where the lists were built for it
  if (E.sym && (want_grad || E.det || !E.img_trg))
    throw Error{PDMK_ERR_UNSUPPORTED, "symmetric residual lists without their evaluation"};
  if constexpr (D == 3 && sizeof(Real) == 8) {
    if (P->o.eps >= 1e-10) {
      if (want_grad) go(k_direct<D, NE, true, Real, 1, false>);
      else if (E.sym) go(k_direct<D, NE, false, Real, 1, true>);
      else go(k_direct<D, NE, false, Real, 1, false>);
      return;
    }
  }
  if (want_grad) go(k_direct<D, NE, true, Real, 2, false>);
  else if (E.sym && sizeof(Real) == 4) go(k_direct_w4<D, NE, false, Real, 2, true>);
  else if (E.sym) go(k_direct<D, NE, false, Real, 2, true>);
  else go(k_direct<D, NE, false, Real, 2, false>);
}

template <int D, class Real>
static void launch_direct_r(const KParams& kp, Eval& E, pdmk_plan* P, hipStream_t s,
                            bool want_grad, unsigned long long* nsup) {
  const bool f32 = sizeof(Real) == 4;
  const int nv = D == 3 ? (f32 ? kp.nE32 : kp.nE) : (f32 ? kp.nF232 : kp.nF2);
  const int nd = D == 3 ? (f32 ? kp.nEd32 : kp.nEd) : (f32 ? kp.nF2d32 : kp.nF2d);
  const int nc = want_grad ? std::max(nv, nd) : nv;
  // Horner pays one FMA per padding term: lengths close to the series'
  if (nc <= 8) launch_direct_t<D, 8, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 10) launch_direct_t<D, 10, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 12) launch_direct_t<D, 12, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 14) launch_direct_t<D, 14, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 16) launch_direct_t<D, 16, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 20) launch_direct_t<D, 20, Real>(kp, E, P, s, want_grad, nsup);
  else if (nc <= 24) launch_direct_t<D, 24, Real>(kp, E, P, s, want_grad, nsup);
  else launch_direct_t<D, 32, Real>(kp, E, P, s, want_grad, nsup);
}

template <int D>
static void launch_direct(const KParams& kp, Eval& E, pdmk_plan* P, hipStream_t s,
                          bool want_grad, unsigned long long* nsup) {
  if (kp.precision == PDMK_PREC_MIXED && (P->mixed_parts & 1))
    launch_direct_r<D, float>(kp, E, P, s, want_grad, nsup);
  else launch_direct_r<D, double>(kp, E, P, s, want_grad, nsup);
}

template <int D, class Real>
static void launch_transfer(const KParams& kp, const Level& Lp, const Level& Lc, int up,
                            const void* src_, void* dst_, pdmk_plan* P, Eval& E,
                            hipStream_t s) {
  if (D == 3 && Lc.nnl > 0 && transfer_mfma<Real>(P, Lp, Lc, up != 0, src_, dst_, E.det, s))
    return;
  const Real* src = static_cast<const Real*>(src_);
  Real* dst = static_cast<Real*>(dst_);
  const int p = kp.p;
  const int pD = D == 3 ? p * p * p : p * p;
  const size_t full = (size_t)(pD + 2 * p * 40) * sizeof(Real);
  const bool lds = full <= 100 * 1024;
  const size_t smem = lds ? full : (size_t)2 * p * 40 * sizeof(Real);
  const int nown = (pD + 255) / 256;
  const int mode = up ? (nown <= 48 ? 0 : 1) : 2;
  const int nblocks = mode == 0 ? Lp.nnl : Lc.nnl;
  Real* scratch = lds ? nullptr : E.alloc<Real>((size_t)nblocks * pD);
  // fixed-order mode: per-child up transfers (mode 1) add one octant per launch
  const bool octs = E.det && mode == 1;
#define PDMK_TR(PM, L, NO, MO)                                                                  \
  do {                                                                                          \
    if (p > PM || (MO == 0 && pD > 256 * NO))                                                   \
      throw Error{PDMK_ERR_UNSUPPORTED, "transfer shape"};                                      \
    ensure_lds((const void*)&k_transfer<D, PM, L, NO, MO, Real>, smem);                         \
    for (int o = octs ? 0 : -1; o < (octs ? (1 << D) : 0); ++o)                                 \
      hipLaunchKernelGGL((k_transfer<D, PM, L, NO, MO, Real>), dim3(nblocks), dim3(256), smem,  \
                         s, kp, Lp, Lc, src, dst, P->d_Tm, scratch, o);                         \
  } while (0)
  // the line length PMAX must cover p: a shorter one leaves outputs p > PMAX
  // of every line uncomputed
  if (mode == 0) {
    if (nown <= 8) {   // 2D for every order (p <= 40)
      if (p <= 16) PDMK_TR(16, true, 8, 0);
      else if (p <= 24) PDMK_TR(24, true, 8, 0);
      else if (p <= 32) PDMK_TR(32, true, 8, 0);
      else PDMK_TR(40, true, 8, 0);
    } else if (nown <= 24) {   // 3D, p <= 18
      if (p <= 16) PDMK_TR(16, true, 24, 0);
      else PDMK_TR(24, true, 24, 0);
    } else {   // 3D, p <= 23
      if (lds) PDMK_TR(24, true, 48, 0);
      else PDMK_TR(32, false, 48, 0);
    }
  } else {
    const bool m1 = mode == 1;
    if (lds) {
      if (p <= 16) { if (m1) PDMK_TR(16, true, 1, 1); else PDMK_TR(16, true, 1, 2); }
      else if (p <= 24) { if (m1) PDMK_TR(24, true, 1, 1); else PDMK_TR(24, true, 1, 2); }
      else if (p <= 32) { if (m1) PDMK_TR(32, true, 1, 1); else PDMK_TR(32, true, 1, 2); }
      else { if (m1) PDMK_TR(40, true, 1, 1); else PDMK_TR(40, true, 1, 2); }
    } else {
      if (p <= 24) { if (m1) PDMK_TR(24, false, 1, 1); else PDMK_TR(24, false, 1, 2); }
      else if (p <= 32) { if (m1) PDMK_TR(32, false, 1, 1); else PDMK_TR(32, false, 1, 2); }
      else { if (m1) PDMK_TR(40, false, 1, 1); else PDMK_TR(40, false, 1, 2); }
    }
  }
#undef PDMK_TR
}

template <int D, class Real>
static void launch_anterp(const KParams& kp, const Level& L, const Level& C, int l, Eval& E,
                          pdmk_plan* P, hipStream_t s) {
  const int p = kp.p;
  Real* Q = static_cast<Real*>(L.proxy_q);
  if (D == 3 && anterp_mfma<Real>(P, L, C, l, E.sx, E.sq, E.n_img, Q, s)) return;
#define PDMK_AN(PM) \
  hipLaunchKernelGGL((k_anterp<D, PM, Real>), dim3(L.nnl), dim3(256), 0, s, kp, L, C, l, E.sx, \
                     E.sq, E.n_img, P->d_nodes, P->d_bw, Q)
  if (p <= 16) PDMK_AN(16);
  else if (p <= 24) PDMK_AN(24);
  else if (p <= 32) PDMK_AN(32);
  else PDMK_AN(40);
#undef PDMK_AN
}

template <int D, class Real>
static void launch_eval_children(const KParams& kp, const Level& Lp, const Level& Lc, int l,
                                 Eval& E, pdmk_plan* P, hipStream_t s, bool want_grad) {
  const int p = kp.p;
#define PDMK_EV(PM, NT, G)                                                                   \
  hipLaunchKernelGGL((k_eval_children<D, PM, NT, G, Real>), dim3(Lp.nnl), dim3(NT), 0, s, kp, \
                     Lp, Lc, l, E.tx, E.n_trg, P->d_nodes, P->d_bw, E.pot_sorted,             \
                     E.grad_sorted)
  if (want_grad) {
    if (p <= 16) PDMK_EV(16, 64, true);
    else if (p <= 24) PDMK_EV(24, 64, true);
    else if (p <= 32) PDMK_EV(32, 32, true);
    else PDMK_EV(40, 32, true);
  } else {
    if (p <= 16) PDMK_EV(16, 128, false);
    else if (p <= 24) PDMK_EV(24, 128, false);
    else if (p <= 32) PDMK_EV(32, 64, false);
    else PDMK_EV(40, 64, false);
  }
#undef PDMK_EV
}

// LDS bytes of the fused plane-wave kernels for element type Real.
static size_t lds_pw_out(int p, int J, size_t rs) {
  const size_t n1 = 2 * J + 1;
  return (size_t)p * p * p * rs + (2 * n1 * p + (size_t)p * p + n1 * p) * 2 * rs;
}
static size_t lds_pw_in(int p, int J, size_t rs) {
  const size_t n1 = 2 * J + 1;
  return (size_t)p * p * p * rs + (n1 * p + n1 * n1 + n1 * p + (size_t)p * p) * 2 * rs;
}

// Near-field pipeline with proxy and plane-wave data of type Real.  Real =
// float is used only with the fused 3D plane-wave kernels; the generic
// axis-by-axis path (2D, or tensors too large for LDS) is FP64.
template <int D, class Real>
static void near_impl(pdmk_plan* P, Eval& E, bool want_grad) {
  using C = Cx<Real>;
  const KParams& kp = P->kp;
  hipStream_t s = E.s;
  const int p = kp.p, J = kp.J;
  const int pD = D == 3 ? p * p * p : p * p;
  const int n1 = 2 * J + 1;
  const int nlev = (int)E.lev.size();
  const bool tm = E.timing;   // per-stage events (not inside a kept-tree execute)
  if (tm)
    for (auto& e : E.near_ev) e = E.event();
  E.near_pending = tm;
  hipEvent_t e0 = E.near_ev[0], e1 = E.near_ev[1], e2 = E.near_ev[2], e3 = E.near_ev[3];
  // [0] colleague pairs translated, [1] boxes given incoming plane waves,
  // [2] residual pairs inside the support
  // (cnt[3]: staged pairs; cnt[4 ...]: the residual sums' statistic slots,
  // then the colleague translation's, folded into cnt[0], cnt[1])
  const int ncnt = 4 + 2 * kStatSlots + 2 * kTransSlots;
  unsigned long long* cnt = E.alloc<unsigned long long>(ncnt);
  fill_zero(cnt, ncnt * sizeof(unsigned long long), s);
  unsigned long long* nsup = cnt + 4;
  unsigned long long* trslots = cnt + 4 + 2 * kStatSlots;
  fill_zero(E.pot_sorted, sizeof(double) * E.n_trg, s);
  if (want_grad)
    fill_zero(E.grad_sorted, sizeof(double) * E.n_trg * D, s);
  if (tm) PDMK_HIP(hipEventRecord(e0, s));
  // residual sums (add into the zeroed pot_sorted)
  if (E.nitems > 0) launch_direct<D>(kp, E, P, s, want_grad, nsup);
  if (tm) PDMK_HIP(hipEventRecord(e1, s));
  // proxies
  int maxnl = 0;
  for (int l = 0; l < nlev; ++l) maxnl = std::max(maxnl, E.lev[l].nnl);
  // matrix-core plane waves: the incoming kernel writes every proxy potential
  // (zeros for boxes without targets), so only the other paths clear them
  const bool mfma = D == 3 && P->pw_mfma && pw_mfma_shape(p, J, sizeof(Real)).ok;
  for (int l = 0; l < nlev; ++l) {
    Level& L = E.lev[l];
    if (L.nnl == 0) continue;
    // 64 entries of zero padding: the leaf evaluation reads whole register
    // rows past the last tensor entry
    L.proxy_q = E.alloc<Real>((size_t)L.nnl * pD + 64);
    L.proxy_phi = E.alloc<Real>((size_t)L.nnl * pD + 64);
    if (mfma)
      fill_zero(static_cast<Real*>(L.proxy_phi) + (size_t)L.nnl * pD, sizeof(Real) * 64, s);
    else
      fill_zero(L.proxy_phi, sizeof(Real) * ((size_t)L.nnl * pD + 64), s);
  }
  if (maxnl > 0) {
    // upward pass
    for (int l = nlev - 2; l >= 0; --l) {
      Level& L = E.lev[l];
      if (L.nnl == 0) continue;
      Level& Cl = E.lev[l + 1];
      launch_anterp<D, Real>(kp, L, Cl, l, E, P, s);
      if (Cl.nnl > 0) launch_transfer<D, Real>(kp, L, Cl, 1, Cl.proxy_q, L.proxy_q, P, E, s);
    }
    // plane waves, level by level
    const int64_t s1 = (int64_t)(J + 1) * p * (D == 3 ? p : 1);
    const int64_t s2 = D == 3 ? (int64_t)(J + 1) * n1 * p : 0;
    const int64_t s3 = D == 3 ? (int64_t)(J + 1) * n1 * n1 : (int64_t)(J + 1) * n1;
    const size_t lds_out = lds_pw_out(p, J, sizeof(Real));
    const size_t lds_in = lds_pw_in(p, J, sizeof(Real));
    const bool fused = D == 3 && lds_out <= 150 * 1024 && lds_in <= 150 * 1024;
    // matrix-core path: outgoing and translated incoming expansions in compact
    // half-ball order; vector-ALU path: outgoing expansions on the full grid.
    // Axis-by-axis path (neither fused nor matrix-core, FP64): library GEMMs
    // for the contractions where the call may allocate (the proxy tensors go
    // through one complex staging buffer of p^d per box); in 3D the
    // expansions are then kept in compact half-ball order too and translated
    // by the matrix-core path's kernel
    const bool gemm = E.lib_gemm && !mfma && !fused && sizeof(Real) == 8;
    const bool compact = mfma || (gemm && D == 3);
    C* bS = E.alloc<C>((size_t)maxnl * (compact ? P->nball : s3));
    C* bIw = compact ? E.alloc<C>((size_t)maxnl * P->nball) : nullptr;
    // axis-by-axis path: the intermediate tensors of at most `chunk` boxes at a
    // time (about 2 GB), so that their size does not grow with the level (at
    // p = 40 they take 3.9 MB per box); only the outgoing plane waves, which
    // the translation reads across colleagues, are kept for the whole level
    const int64_t per_box = (s1 + s2 + s3 + (gemm ? pD : 0)) * (int64_t)sizeof(double2);
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(maxnl, (2ll << 30) / per_box));
    double2* bA = fused ? nullptr : E.alloc<double2>((size_t)chunk * s1);
    double2* bB = (D == 3 && !fused) ? E.alloc<double2>((size_t)chunk * s2) : nullptr;
    double2* bI = fused ? nullptr : E.alloc<double2>((size_t)chunk * s3);
    double2* bQ = gemm ? E.alloc<double2>((size_t)chunk * pD) : nullptr;
    unsigned long long* npairs = cnt;
    E.pw_split = mfma;
    const C* Ftab = reinterpret_cast<const C*>(sizeof(Real) == 4 ? (const void*)P->d_Ff
                                                                 : (const void*)P->d_F);
    if (fused) {
      ensure_lds((const void*)&k_pw_out<Real>, lds_out);
      ensure_lds((const void*)&k_pw_in<Real>, lds_in);
    }
    for (int l = 0; l < nlev; ++l) {
      Level& L = E.lev[l];
      if (L.nnl == 0) continue;
      const int nn = L.nnl;
      const double h = kp.rc / (double)(1 << l);
      const double levfac = D == 3 ? 1.0 / (3.0 * h) : 1.0;
      const int zz = D == 3 ? p : 1;
      // pe[0] | outgoing | pe[1] | translation (matrix-core path) | pe[3] | incoming | pe[2]
      hipEvent_t pe[4] = {nullptr, nullptr, nullptr, nullptr};
      if (tm) {
        for (auto& e : pe) e = E.event();
        E.pw_ev.push_back({pe[0], pe[1], pe[2], pe[3]});
      }
      E.st.n_pwout_boxes += nn;
      if (tm) PDMK_HIP(hipEventRecord(pe[0], s));
      if (mfma) {
        pw_mfma_level<Real>(P, L, nn, L.proxy_q, bS, bIw, L.proxy_phi, levfac, trslots, pe[1],
                            pe[3], s);
        if (tm) PDMK_HIP(hipEventRecord(pe[2], s));
        continue;
      }
      if (fused) {
        hipLaunchKernelGGL(k_pw_out<Real>, dim3(nn), dim3(256), lds_out, s, kp, L,
                           static_cast<const Real*>(L.proxy_q), Ftab, bS);
        if (tm) PDMK_HIP(hipEventRecord(pe[1], s));
        hipLaunchKernelGGL(k_pw_in<Real>, dim3(nn), dim3(256), lds_in, s, kp, L, bS, Ftab,
                           P->d_dtab, levfac, static_cast<Real*>(L.proxy_phi), npairs);
        if (tm) PDMK_HIP(hipEventRecord(pe[2], s));
        continue;
      }
      if (tm) PDMK_HIP(hipEventRecord(pe[1], s));
      if (sizeof(Real) != 8) throw Error{PDMK_ERR_UNSUPPORTED, "FP32 proxies need the fused path"};
      double2* bSd = reinterpret_cast<double2*>(bS);
      const double* pq = static_cast<const double*>(L.proxy_q);
      double* pphi = static_cast<double*>(L.proxy_phi);
      if (gemm) {
        const double2* F = P->d_F;
        const double2* Fc = P->d_Fc;
        for (int k0 = 0; k0 < nn; k0 += chunk) {
          const int nc = std::min(chunk, nn - k0);
          hipLaunchKernelGGL(k_real_to_cplx, dim3(nblk((int64_t)nc * pD, 256)), dim3(256), 0, s,
                             (int64_t)nc * pD, pq + (int64_t)k0 * pD, bQ);
          axis_gemm(P, s, nc, p, p, zz, 0, J + 1, bQ, bA, F, Fc, J, p, 0, 0);
          if (D == 3) {
            axis_gemm(P, s, nc, J + 1, p, p, 1, n1, bA, bB, F, Fc, 0, p, 0, 0);
            axis_gemm(P, s, nc, J + 1, n1, p, 2, n1, bB, bI, F, Fc, 0, p, 0, 0);
            hipLaunchKernelGGL(k_gather_ball, dim3(nblk((int64_t)nc * P->nball, 256)),
                               dim3(256), 0, s, nc, P->nball, J, P->d_ball, (const double2*)bI,
                               bSd + (int64_t)k0 * P->nball);
          } else {
            axis_gemm(P, s, nc, J + 1, p, 1, 1, n1, bA, bSd + (int64_t)k0 * s3, F, Fc, 0, p, 0,
                      0);
          }
        }
        if (D == 3)
          pw_translate(P, L, bSd, reinterpret_cast<double2*>(bIw), levfac, trslots, s);
        for (int k0 = 0; k0 < nn; k0 += chunk) {
          const int nc = std::min(chunk, nn - k0);
          if (D == 3)
            hipLaunchKernelGGL(k_scatter_ball, dim3(nblk((int64_t)nc * s3, 256)), dim3(256), 0,
                               s, nc, k0, L, P->nball, J, P->d_brow,
                               (const double2*)reinterpret_cast<double2*>(bIw), bI);
          else
            hipLaunchKernelGGL(k_translate<D>, dim3(nblk((int64_t)nc * s3, 256)), dim3(256), 0,
                               s, L, J, k0, nc, bSd, bI, P->d_dtab, levfac, npairs);
          if (D == 3) {
            axis_gemm(P, s, nc, J + 1, n1, n1, 2, p, bI, bB, F, Fc, 0, p, 1, 1);
            axis_gemm(P, s, nc, J + 1, n1, p, 1, p, bB, bA, F, Fc, 0, p, 1, 1);
          } else {
            axis_gemm(P, s, nc, J + 1, n1, 1, 1, p, bI, bA, F, Fc, 0, p, 1, 1);
          }
          // last axis with the Hermitian weights (1 for j = 0, 2 for j > 0),
          // real part added to the proxy potentials
          axis_gemm(P, s, nc, J + 1, p, zz, 0, p, bA, bQ, P->d_Fw, P->d_Fw, J, p, 1, 0);
          hipLaunchKernelGGL(k_add_real, dim3(nblk((int64_t)nc * pD, 256)), dim3(256), 0, s,
                             (int64_t)nc * pD, (const double2*)bQ, pphi + (int64_t)k0 * pD);
        }
        if (tm) PDMK_HIP(hipEventRecord(pe[2], s));
        continue;
      }
      // outgoing: proxy charges -> plane waves (Hermitian half on axis 0)
      for (int k0 = 0; k0 < nn; k0 += chunk) {
        const int nc = std::min(chunk, nn - k0);
        double2* out = bSd + (int64_t)k0 * s3;
        hipLaunchKernelGGL((k_axis<false, 0>), dim3(nblk((int64_t)nc * s1, 256)), dim3(256), 0,
                           s, nc, p, p, zz, 0, J + 1, (const void*)(pq + (int64_t)k0 * pD),
                           (void*)bA, P->d_F, J, p, 0, 0);
        if (D == 3) {
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s2, 256)), dim3(256), 0,
                             s, nc, J + 1, p, p, 1, n1, (const void*)bA, (void*)bB, P->d_F, 0, p,
                             0, 0);
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s3, 256)), dim3(256), 0,
                             s, nc, J + 1, n1, p, 2, n1, (const void*)bB, (void*)out, P->d_F, 0,
                             p, 0, 0);
        } else {
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s3, 256)), dim3(256), 0,
                             s, nc, J + 1, p, 1, 1, n1, (const void*)bA, (void*)out, P->d_F, 0,
                             p, 0, 0);
        }
      }
      for (int k0 = 0; k0 < nn; k0 += chunk) {
        const int nc = std::min(chunk, nn - k0);
        // translation between colleagues with the difference-kernel multiplier
        hipLaunchKernelGGL(k_translate<D>, dim3(nblk((int64_t)nc * s3, 256)), dim3(256), 0, s,
                           L, J, k0, nc, bSd, bI, P->d_dtab, levfac, npairs);
        // incoming: plane waves -> proxy potentials
        if (D == 3) {
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s2, 256)), dim3(256), 0,
                             s, nc, J + 1, n1, n1, 2, p, (const void*)bI, (void*)bB, P->d_F, 0,
                             p, 1, 1);
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s1, 256)), dim3(256), 0,
                             s, nc, J + 1, n1, p, 1, p, (const void*)bB, (void*)bA, P->d_F, 0, p,
                             1, 1);
        } else {
          hipLaunchKernelGGL((k_axis<true, 0>), dim3(nblk((int64_t)nc * s1, 256)), dim3(256), 0,
                             s, nc, J + 1, n1, 1, 1, p, (const void*)bI, (void*)bA, P->d_F, 0, p,
                             1, 1);
        }
        hipLaunchKernelGGL((k_axis<true, 1>), dim3(nblk((int64_t)nc * pD, 256)), dim3(256), 0,
                           s, nc, J + 1, p, zz, 0, p, (const void*)bA,
                           (void*)(pphi + (int64_t)k0 * pD), P->d_F, J, p, 1, 1);
      }
      if (tm) PDMK_HIP(hipEventRecord(pe[2], s));
    }
    // downward pass: parent proxy potential -> non-leaf child proxy potential
    for (int l = 1; l < nlev; ++l) {
      Level& Cl = E.lev[l];
      Level& L = E.lev[l - 1];
      if (Cl.nnl == 0) continue;
      launch_transfer<D, Real>(kp, L, Cl, 0, L.proxy_phi, Cl.proxy_phi, P, E, s);
    }
  }
  if (tm) PDMK_HIP(hipEventRecord(e2, s));
  // leaf targets evaluate their parent's proxy potential
  if (maxnl > 0)
    for (int l = 0; l + 1 < nlev; ++l)
      if (E.lev[l].nnl > 0)
        if (!(D == 3 && eval_leaf_mfma<Real>(P, E.lev[l], E.lev[l + 1], l, E.tx, E.n_trg,
                                             E.pot_sorted, want_grad ? E.grad_sorted : nullptr,
                                             s)))
          launch_eval_children<D, Real>(kp, E.lev[l], E.lev[l + 1], l, E, P, s, want_grad);
  if (tm) {
    PDMK_HIP(hipEventRecord(e3, s));
    // statistics (read only here): the slots folded into cnt[0..3]
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, s, nsup, kStatSlots, cnt + 2, 0);
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, s, trslots, kTransSlots, cnt, 1);
    PDMK_HIP(hipMemcpyAsync(P->h_cnt, cnt, 3 * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
    PDMK_HIP(hipMemcpyAsync(P->h_cnt + 8, cnt + 3, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
  }
}

void near_finish(const pdmk_plan* P, Eval& E) {
  if (!E.near_pending) return;
  E.near_pending = false;
  E.st.n_pw_pairs = (int64_t)P->h_cnt[0];
  E.st.n_pwin_boxes = (int64_t)P->h_cnt[1];
  E.st.n_support_pairs = (int64_t)P->h_cnt[2];
  E.st.n_staged_pairs = (int64_t)P->h_cnt[8];
  E.st.n_direct_pairs = (int64_t)P->h_cnt[3];   // copied by the list stage
  for (auto& pe : E.pw_ev) {
    float a = 0, b = 0, c = 0;
    PDMK_HIP(hipEventElapsedTime(&a, pe[0], pe[1]));
    if (E.pw_split) {
      PDMK_HIP(hipEventElapsedTime(&c, pe[1], pe[3]));
      PDMK_HIP(hipEventElapsedTime(&b, pe[3], pe[2]));
    } else {
      PDMK_HIP(hipEventElapsedTime(&b, pe[1], pe[2]));
    }
    E.st.t_pwout_ms += a;
    E.st.t_pwtr_ms += c;
    E.st.t_pwin_ms += b;
  }
  E.pw_ev.clear();
  float t01, t12, t23;
  PDMK_HIP(hipEventElapsedTime(&t01, E.near_ev[0], E.near_ev[1]));
  PDMK_HIP(hipEventElapsedTime(&t12, E.near_ev[1], E.near_ev[2]));
  PDMK_HIP(hipEventElapsedTime(&t23, E.near_ev[2], E.near_ev[3]));
  E.st.t_direct_ms = t01;
  E.st.t_pw_ms = t12;
  E.st.t_proxy_ms = t23;
}

void stage_near(pdmk_plan* P, Eval& E, bool want_grad) {
  E.pot_sorted = E.alloc<double>(E.n_trg);
  E.grad_sorted = want_grad ? E.alloc<double>(E.n_trg * P->kp.dim) : nullptr;
  const KParams& kp = P->kp;
  const bool f32 = kp.precision == PDMK_PREC_MIXED && (P->mixed_parts & 2) && kp.dim == 3 &&
                   lds_pw_out(kp.p, kp.J, 4) <= 150 * 1024 &&
                   lds_pw_in(kp.p, kp.J, 4) <= 150 * 1024;
  if (kp.dim == 3) {
    if (f32) near_impl<3, float>(P, E, want_grad);
    else near_impl<3, double>(P, E, want_grad);
  } else {
    near_impl<2, double>(P, E, want_grad);
  }
}

}  // namespace pdmk
