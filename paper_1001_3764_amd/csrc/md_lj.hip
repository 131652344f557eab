// Truncated Lennard-Jones forces over the cell stencil (Section 3.2, Eq. 2) for gfx950.
//
// Pair force as in the paper's inner loop: with r2inv = 1/r^2 and r6inv = r2inv^3,
// F_i += (x_i - x_j) * r2inv * r6inv * (12 ljp2 r6inv - 6 ljp1), ljp2 = 4 eps sigma^12,
// ljp1 = 4 eps sigma^6, counted only for r^2 < rc^2 and pairs more than excl bonds
// apart along a chain.  Every pair is evaluated from both sides (as the paper's
// thread-per-atom kernel does), so each atom's force is a private sum: no atomics,
// and the order of the sum is fixed by the sorted cell lists.
//
// Coordinates come from the sorted payload, relative to the centre of each atom's
// cell.  A neighbour cell at offset (ox, oy, oz) contributes x_j + (ox, oy, oz) * edge
// in the home cell's frame.  Mixed precision keeps these as int32 fixed point
// (2^-25 A), so x_i - x_j is an exact integer rounded once to FP32; FP64 uses doubles.
//
// Kernels:
//   k_lj_atom        one lane per home atom walking the stencil cells (the paper's shape);
//   k_lj_tile        one wavefront per home cell: the cell's atoms are wave-uniform (KMAX
//                    at a time) and the stencil's atoms, listed flat in LDS and filtered
//                    by the box bounding the homes, stream across the lanes 64 at a time;
//                    with LIST the candidates are the cell's neighbour list instead;
//   k_lj_half        the same layout over half the stencil, each pair once, both forces
//                    added to int64 fixed-point accumulators (opt-in);
//   k_nl_build,      neighbour-list builds (Sections 3.1-3.2), per atom and per cell, and
//   k_nl_build_tile, the per-atom list walk.
//   k_lj_nl
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "md_internal.h"

namespace mdk {
namespace {

struct alignas(32) Pay64 {
  double x, y, z, tagbits;
};

__device__ inline int32_t pay_tag(const int4& q) { return q.w; }
__device__ inline int32_t pay_tag(const Pay64& q) { return (int32_t)__double_as_longlong(q.tagbits); }

__device__ inline float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ inline int lane() { return (int)(threadIdx.x & 63); }

// Number of set bits of a wave mask below this lane.
__device__ inline int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---------------------------------------------------------------------------------
// Cross-lane exchanges that need no lane-address register.  A shuffle through
// ds_bpermute takes a per-lane byte address; the compiler computes those once and
// keeps them live for the whole kernel (one register per distinct pattern), which in
// the tile kernel pushed values out to scratch.  These use gfx950's 32- and 16-lane
// row swaps and DPP moves within 16-lane rows, so only the data travels.
//
// Swaps: after v_permlane32_swap(a, b) lanes 32-63 of a hold lanes 0-31 of b and lanes
// 0-31 of b hold lanes 32-63 of a; v_permlane16_swap does the same between the odd
// 16-lane rows of a and the even rows of b.  DPP: row_ror:8 reads lane l ^ 8 (rotation
// by half of a 16-lane row), row_half_mirror lane l ^ 7, quad_perm [2,3,0,1] lane l ^ 2
// and [1,0,3,2] lane l ^ 1.

enum class Xl { Swap32, Swap16, Ror8, Mirror8, Quad2, Quad1 };

__device__ __forceinline__ uint32_t dpp32(uint32_t x, Xl p) {
  switch (p) {
    case Xl::Ror8: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xf, 0xf, false);
    case Xl::Mirror8: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xf, 0xf, false);
    case Xl::Quad2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4e, 0xf, 0xf, false);
    default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xb1, 0xf, 0xf, false);
  }
}

// Lanes below the split (l & 32, or l & 16, clear) get a[l] and a[partner]; lanes above
// get b[partner] and b[l].  Returned as {first, second}: first + second is the pair sum
// each side keeps.
__device__ __forceinline__ void swap32(uint32_t a, uint32_t b, Xl p, uint32_t& first, uint32_t& second) {
  if (p == Xl::Swap32) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    first = r[0];
    second = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    first = r[0];
    second = r[1];
  }
}

template <typename T>
struct XlBits;
template <>
struct XlBits<float> {
  static constexpr int n = 1;
  __device__ static void split(float x, uint32_t* w) { w[0] = __float_as_uint(x); }
  __device__ static float join(const uint32_t* w) { return __uint_as_float(w[0]); }
};
template <>
struct XlBits<double> {
  static constexpr int n = 2;
  __device__ static void split(double x, uint32_t* w) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    w[0] = (uint32_t)b;
    w[1] = (uint32_t)(b >> 32);
  }
  __device__ static double join(const uint32_t* w) {
    return __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
  }
};
template <>
struct XlBits<int> {
  static constexpr int n = 1;
  __device__ static void split(int x, uint32_t* w) { w[0] = (uint32_t)x; }
  __device__ static int join(const uint32_t* w) { return (int)w[0]; }
};

// Sum kept by each side of a swap exchange: lanes below the split get a[l] + a[partner],
// lanes above b[partner] + b[l] (the halving step of a reduction of two value sets).
template <typename T>
__device__ __forceinline__ T swap_sum(T a, T b, Xl p) {
  uint32_t wa[XlBits<T>::n], wb[XlBits<T>::n], f[XlBits<T>::n], s[XlBits<T>::n];
  XlBits<T>::split(a, wa);
  XlBits<T>::split(b, wb);
#pragma unroll
  for (int i = 0; i < XlBits<T>::n; ++i) swap32(wa[i], wb[i], p, f[i], s[i]);
  return XlBits<T>::join(f) + XlBits<T>::join(s);
}

// The value of x on the partner lane (l ^ 32, l ^ 16, l ^ 8, l ^ 7, l ^ 2 or l ^ 1).
template <typename T>
__device__ __forceinline__ T partner(T x, Xl p) {
  uint32_t w[XlBits<T>::n], o[XlBits<T>::n];
  XlBits<T>::split(x, w);
  if (p == Xl::Swap32 || p == Xl::Swap16) {
    const bool above = (lane() & (p == Xl::Swap32 ? 32 : 16)) != 0;
#pragma unroll
    for (int i = 0; i < XlBits<T>::n; ++i) {
      uint32_t f, s;
      swap32(w[i], w[i], p, f, s);
      o[i] = above ? f : s;
    }
  } else {
#pragma unroll
    for (int i = 0; i < XlBits<T>::n; ++i) o[i] = dpp32(w[i], p);
  }
  return XlBits<T>::join(o);
}

// x + x[l ^ mask]; both lanes of a pair add the same two values, so they agree bitwise.
template <typename T>
__device__ __forceinline__ T pair_add(T x, Xl p) {
  if (p == Xl::Swap32 || p == Xl::Swap16) return swap_sum(x, x, p);
  return x + partner(x, p);
}

// The butterfly patterns from the widest down; masks 32, 16, 8, 7, 2, 1 span all six
// lane bits, so after levels [from, 6) every lane of a 2^(6 - from)-lane group holds the
// group's sum (the same value on each).
constexpr Xl kLevel[6] = {Xl::Swap32, Xl::Swap16, Xl::Ror8, Xl::Mirror8, Xl::Quad2, Xl::Quad1};

template <typename T>
__device__ __forceinline__ T group_sum(T x, int from) {
#pragma unroll
  for (int lv = from; lv < 6; ++lv) x = pair_add(x, kLevel[lv]);
  return x;
}

// Relative half-width of the band around rc^2 decided in FP64 (well above the FP32 error
// of r^2 from exact fixed-point differences, ~3e-7, plus the 2^-26 A position rounding).
constexpr double kBand = 1e-6;
// Close contacts (r < kCloseSigma sigma, where the pair force exceeds ~50 kcal/mol/A for the
// polyethylene parameters) are evaluated in FP64 (see Band).
constexpr double kCloseSigma = 0.75;
constexpr int kBandQueue = 64;   // band pairs a tile wave queues per home group
constexpr int kBandSteps = 8;    // candidate steps with band pairs a tile wave records per group

// Values that are the same on every lane, moved to scalar registers.
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline double uni(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The value of x on lane k (k wave-uniform), in scalar registers.
__device__ inline int lane_value(int x, int k) { return __builtin_amdgcn_readlane(x, k); }
__device__ inline double lane_value(double x, int k) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Minimum and maximum over lanes [0, K) (K = 1, 2, 4, 8 or 16; the other lanes of the first
// 16-lane row hold the neutral element), as a vector-register value on every lane: a
// butterfly over lane bits 0-3 within the row (xor 1, xor 2, the half-row mirror, xor 8), then
// lane 0's result moved to every lane.
template <typename T>
__device__ inline T box_top();
template <>
__device__ inline int box_top<int>() { return 0x7fffffff; }
template <>
__device__ inline double box_top<double>() { return __builtin_huge_val(); }

template <typename T>
__device__ __forceinline__ T in_vgpr(T x) {
  if constexpr (std::is_same<T, int>::value) asm volatile("" : "+v"(x));
  return x;
}

template <int K, bool MAX, typename T>
__device__ __forceinline__ T first_lanes_ext(T x) {
  constexpr Xl lv[4] = {Xl::Quad1, Xl::Quad2, Xl::Mirror8, Xl::Ror8};
#pragma unroll
  for (int l = 0; (1 << l) < K; ++l) {
    const T y = partner(x, lv[l]);
    x = MAX ? max(x, y) : min(x, y);
  }
  return in_vgpr(lane_value(x, 0));
}
template <int K, typename T>
__device__ __forceinline__ T first_lanes_min(T x) { return first_lanes_ext<K, false>(x); }
template <int K, typename T>
__device__ __forceinline__ T first_lanes_max(T x) { return first_lanes_ext<K, true>(x); }

template <typename P>
struct LjPair {
  P f12[4], f6[4], e12[4], e6[4], ecut[4];
  P f12_fold;               // f12[0] / f6[0] (one type pair: the force factor's inline constant)
  float band_lo, band_hi;   // the cutoff band (see Band), computed once on the host
  float close;              // close-contact bound (see Band), computed once on the host
};

template <typename P>
__device__ inline P pick(const P* a, int t) {
  return t == 0 ? a[0] : (t == 1 ? a[1] : (t == 2 ? a[2] : a[3]));
}

// The two ends of the FP32 pair range, in the fixed-point units of r2s (2^-50 A^2).
// Cutoff band: the FP32 path counts a pair as inside when r2s < hi.  Pairs with
// lo <= r2s < hi are in the band: there the FP32 r^2 cannot tell the side of the cutoff, so
// each is re-decided in FP64 and, if the FP64 test puts it outside, its force is taken back
// out (remove_band_pair).
// Close contacts: pairs with r2s < close (r below kCloseSigma times the smallest LJ sigma)
// never enter the FP32 sums.  Their force grows as r^-13 and FP32's few-ulp relative error
// on it would exceed 1e-5 of the RMS force (a contact at 2.0 A in a grown melt carries
// ~80 times the RMS force); each is evaluated in FP64 from the FP64 positions instead and
// added to its home's force (add_close_pair).  They are rare in a melt.
struct Band {
  float lo, hi, close;
};
template <typename P>
__device__ inline Band band_of(const LjPair<P>& c) {
  return Band{c.band_lo, c.band_hi, c.close};
}
__device__ __forceinline__ bool in_band(float r2s, bool keep, const Band& b) {
  return keep && r2s >= b.lo && r2s < b.hi;
}
__device__ __forceinline__ bool is_close(float r2s, bool keep, const Band& b) { return keep && r2s < b.close; }

// Exact cutoff test for a band pair (about one candidate in 10^6): r^2 < rc^2 decided from
// the FP64 positions with the operation order of a plain FP64 evaluation (no fused
// multiply-add), so the pair set is the FP64 one.  The image shift uses t * (1/L); it can
// differ from rint(t / L) only for |t| ~ L/2, i.e. |d| ~ L/2 >= 1.5 rc, never for a pair
// near the cutoff.  Returns the minimum-image difference and r^2.
__device__ __forceinline__ bool inside_cutoff_f64(const double* __restrict__ pos, int64_t n, const BoxDev& B,
                                                  int32_t i, int32_t j, double rc2, double (&d)[3], double& r2) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double t = __dadd_rn(pos[q * n + i], -pos[q * n + j]);
    d[q] = __dadd_rn(t, -__dmul_rn(B.L[q], rint(__dmul_rn(t, B.invL[q]))));
    r2 = q == 0 ? __dmul_rn(d[q], d[q]) : __dadd_rn(r2, __dmul_rn(d[q], d[q]));
  }
  return r2 < rc2;
}

// Takes a band pair that the FP64 test puts outside back out of accumulators in units of
// 2^25.  The pair sits at r ~ rc, where the force is ~|F(rc)|; evaluating it from the
// FP64 difference instead of the fixed-point one leaves a residue ~1e-7 of that.
template <bool ENERGY>
__device__ __forceinline__ void remove_band_pair(const double (&d)[3], double r2, float f12, float f6, float e12,
                                                 float e6, float ecut, float& ax, float& ay, float& az, double& e,
                                                 double& es, double& w) {
  const float r2i = 1.0f / (float)r2;
  const float r6 = r2i * r2i * r2i;
  const float g = r6 * (f12 * r6 - f6);
  const float ffs = g * r2i * (float)kFix;
  ax -= ffs * (float)d[0];
  ay -= ffs * (float)d[1];
  az -= ffs * (float)d[2];
  if (ENERGY) {
    const float en = r6 * (e12 * r6 - e6);
    e -= (double)en;
    es -= (double)en - (double)ecut;
    w -= (double)g;
  }
}

// Adds a close contact to FP64 accumulators (kcal/mol/A): the force from the FP64
// minimum-image difference d = x_i - x_j, in a plain FP64 operation order.
template <bool ENERGY>
__device__ __forceinline__ void add_close_pair(const double (&d)[3], double r2, double f12, double f6, double e12,
                                               double e6, double ecut, double& cx, double& cy, double& cz,
                                               double& e, double& es, double& w) {
  const double r2i = 1.0 / r2;
  const double r6 = r2i * r2i * r2i;
  const double g = r6 * (f12 * r6 - f6);
  const double ffs = g * r2i;
  cx += ffs * d[0];
  cy += ffs * d[1];
  cz += ffs * d[2];
  if (ENERGY) {
    const double en = r6 * (e12 * r6 - e6);
    e += en;
    es += en - ecut;
    w += g;
  }
}

// x clamped to [lo, hi] (lo <= hi), for the bounding-box filter.  Fixed point: the median
// of the three in one instruction (the compiler cannot prove lo <= hi, and a max and a min
// are two); FP64: a max and a min.
__device__ __forceinline__ int clamp_box(int x, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}
__device__ __forceinline__ double clamp_box(double x, double lo, double hi) { return min(max(x, lo), hi); }

// FP32 r^2 of an exact fixed-point difference (units of 2^-50 A^2).  Written with explicit
// fused multiply-adds so that every call site rounds identically.
__device__ __forceinline__ float r2_fix(float dx, float dy, float dz) {
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// One pair, mixed precision.  d* are exact fixed-point differences x_i - x_j; the force
// accumulated in a* is in units of 2^25 (the caller scales the final sum by 2^-25).
// Pairs in the cutoff band are counted; bmax keeps the bits of the largest r2s counted
// (r2s >= 0, so integer order is float order), so that the caller sees a band pair
// (bmax >= lo) at one integer max per pair and settles it.  A close contact (r2s < close)
// is not counted: near is set, and the caller evaluates it in FP64.
// Returns r2s.  BRANCHLESS evaluates the force for every lane and zeroes it outside.
// FOLD: f12 holds f12 / f6 and the caller multiplies the summed force by f6 (one type
// pair: the force factor is then one FMA with an inline constant and no register copy).
template <bool ENERGY, bool BRANCHLESS, bool FOLD = false>
__device__ __forceinline__ float pair_fix(int dqx, int dqy, int dqz, bool keep, const Band& bd, float f12,
                                          float f6, float e12, float e6, float ecut, float& ax, float& ay,
                                          float& az, double& e, double& es, double& w, int32_t& bmax,
                                          bool& near) {
  const float dx = (float)dqx, dy = (float)dqy, dz = (float)dqz;
  const float r2s = r2_fix(dx, dy, dz);
  const bool lt_close = r2s < bd.close;   // one compare serves both masks
  const bool kh = keep && r2s < bd.hi;
  near = near || (kh && lt_close);
  const bool hit = kh && !lt_close;
  if (BRANCHLESS || hit) {
    const float r2 = r2s * kInvFix2F;
    const float r2i = rcp_f(r2);
    const float r6 = r2i * r2i * r2i;
    const float g = FOLD ? r6 * __builtin_fmaf(f12, r6, -1.0f) : r6 * (f12 * r6 - f6);   // F . r (/ f6)
    float ffs = g * r2i;
    if (BRANCHLESS) ffs = hit ? ffs : 0.0f;
    ax += ffs * dx;
    ay += ffs * dy;
    az += ffs * dz;
    bmax = max(bmax, __float_as_int(BRANCHLESS ? (hit ? r2s : 0.0f) : r2s));
    if (ENERGY && hit) {
      const float en = r6 * (e12 * r6 - e6);
      e += (double)en;
      es += (double)en - (double)ecut;
      w += (double)(FOLD ? g * f6 : g);
    }
  }
  return r2s;
}

// One pair, FP64.
template <bool ENERGY>
__device__ __forceinline__ void pair_f64(double dx, double dy, double dz, bool keep, double rc2, double f12,
                                         double f6, double e12, double e6, double ecut, double& ax, double& ay,
                                         double& az, double& e, double& es, double& w) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (keep && r2 < rc2) {
    const double r2i = 1.0 / r2;
    const double r6 = r2i * r2i * r2i;
    const double g = r6 * (f12 * r6 - f6);
    const double ffs = g * r2i;
    ax += ffs * dx;
    ay += ffs * dy;
    az += ffs * dz;
    if (ENERGY) {
      const double en = r6 * (e12 * r6 - e6);
      e += en;
      es += en - ecut;
      w += g;
    }
  }
}

template <int NW>
__device__ void block_energy(double e, double es, double w, dd (*red)[3], dd* out) {
  dd q[3] = {dd_from(0.5 * e), dd_from(0.5 * es), dd_from(0.5 * w)};
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int lv = 0; lv < 6; ++lv) q[k] = dd_add(q[k], dd{partner(q[k].hi, kLevel[lv]), partner(q[k].lo, kLevel[lv])});
  if (lane() == 0)
    for (int k = 0; k < 3; ++k) red[threadIdx.x >> 6][k] = q[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      dd s = red[0][k];
      for (int wv = 1; wv < NW; ++wv) s = dd_add(s, red[wv][k]);
      out[k] = s;
    }
}

// ---------------------------------------------------------------------------------
// Lane per home atom: slot s of the sorted arrays is one lane; the lane walks the
// (2R+1)^3 cells around its own cell.
template <bool FP64, bool ENERGY>
__global__ __launch_bounds__(kLjAtomBlock) void k_lj_atom(Views v, FFDev ff, LjPair<float> cf,
                                                          LjPair<double> cd) {
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using P = std::conditional_t<FP64, double, float>;
  __shared__ dd red[kLjAtomBlock / 64][3];
  const int b = v.lj_blk_box[blockIdx.x];
  const BoxDev& B = v.boxes[b];
  const int local = ((int)blockIdx.x - B.lj_blk_off) * kLjAtomBlock + (int)threadIdx.x;
  const bool active = local < B.n_atoms;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);
  const int32_t* __restrict__ cstart = v.cell_start;
  const int R = v.R;
  const Band bd = band_of(cf);
  double e = 0.0, es = 0.0, w = 0.0;
  if (active) {
    const int64_t s = (int64_t)B.atom_off + local;
    const PayT pi = pay[s];
    const int32_t tag = pay_tag(pi);
    const int32_t i = tag_index(tag);
    const int ti = tag_type(tag);
    const int32_t cs = chain_first(i, ff);
    const int32_t lo = max(i - ff.excl, cs);
    const int32_t hi = min(i + ff.excl, cs + ff.chain_len - 1);
    const uint32_t span = (uint32_t)(hi - lo);
    const int c = v.scell[s] - B.cell_off;
    const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
    const Cell3 k3 = cell_coords(c, B);
    const int kx = k3.x, ky = k3.y, kz = k3.z;
    P fx = 0, fy = 0, fz = 0;
    double cx = 0.0, cy = 0.0, cz = 0.0;   // close contacts (mixed), FP64
    for (int oz = -R; oz <= R; ++oz) {
      int nz = kz + oz;
      nz += nz < 0 ? M2 : 0;
      nz -= nz >= M2 ? M2 : 0;
      for (int oy = -R; oy <= R; ++oy) {
        int ny = ky + oy;
        ny += ny < 0 ? M1 : 0;
        ny -= ny >= M1 ? M1 : 0;
        for (int ox = -R; ox <= R; ++ox) {
          int nx = kx + ox;
          nx += nx < 0 ? M0 : 0;
          nx -= nx >= M0 ? M0 : 0;
          const int nc = B.cell_off + nx + M0 * (ny + M1 * nz);
          const int t1 = cstart[nc + 1];
          // home position in the frame of the neighbour cell: x_i - (ox, oy, oz) * edge
          if constexpr (FP64) {
            const double hx = pi.x - ox * B.edge[0], hy = pi.y - oy * B.edge[1], hz = pi.z - oz * B.edge[2];
            for (int t = cstart[nc]; t < t1; ++t) {
              const PayT pj = pay[t];
              const int32_t tj = pay_tag(pj);
              const bool keep = (uint32_t)(tag_index(tj) - lo) > span;
              const int tt = ff.uniform_lj ? 0 : ti * 2 + tag_type(tj);
              pair_f64<ENERGY>(hx - pj.x, hy - pj.y, hz - pj.z, keep, ff.rc2, pick(cd.f12, tt), pick(cd.f6, tt),
                               pick(cd.e12, tt), pick(cd.e6, tt), pick(cd.ecut, tt), fx, fy, fz, e, es, w);
            }
          } else {
            const int hx = pi.x - ox * B.edge_q[0], hy = pi.y - oy * B.edge_q[1], hz = pi.z - oz * B.edge_q[2];
            for (int t = cstart[nc]; t < t1; ++t) {
              const PayT pj = pay[t];
              const int32_t tj = pay_tag(pj);
              const bool keep = (uint32_t)(tag_index(tj) - lo) > span;
              const int tt = ff.uniform_lj ? 0 : ti * 2 + tag_type(tj);
              int32_t bmax = 0;
              bool near = false;
              const float r2s = pair_fix<ENERGY, false>(hx - pj.x, hy - pj.y, hz - pj.z, keep, bd, pick(cf.f12, tt),
                                                        pick(cf.f6, tt), pick(cf.e12, tt), pick(cf.e6, tt),
                                                        pick(cf.ecut, tt), fx, fy, fz, e, es, w, bmax, near);
              double d[3], r2;
              if (in_band(r2s, keep, bd) && !inside_cutoff_f64(v.pos, v.N, B, i, tag_index(tj), ff.rc2, d, r2))
                remove_band_pair<ENERGY>(d, r2, pick(cf.f12, tt), pick(cf.f6, tt), pick(cf.e12, tt),
                                         pick(cf.e6, tt), pick(cf.ecut, tt), fx, fy, fz, e, es, w);
              if (near) {   // rare: a close contact, in FP64
                inside_cutoff_f64(v.pos, v.N, B, i, tag_index(tj), ff.rc2, d, r2);
                add_close_pair<ENERGY>(d, r2, pick(cd.f12, tt), pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt),
                                       pick(cd.ecut, tt), cx, cy, cz, e, es, w);
              }
            }
          }
        }
      }
    }
    if constexpr (!FP64) {
      fx = (float)((double)fx * (double)kInvFixF + cx);
      fy = (float)((double)fy * (double)kInvFixF + cy);
      fz = (float)((double)fz * (double)kInvFixF + cz);
    }
    P* f = static_cast<P*>(v.f_lj);
    f[i] = fx;
    f[v.N + i] = fy;
    f[2 * v.N + i] = fz;
  }
  if (ENERGY) block_energy<kLjAtomBlock / 64>(e, es, w, red, v.part_lj + (int64_t)blockIdx.x * 3);
}

// ---------------------------------------------------------------------------------
// Cell tile: one wave per home cell.  The wave lists its (2R+1)^3 stencil once, as a flat
// array of candidates in LDS (sorted-array index << 7 | stencil offset code), and streams
// that list 64 lanes at a time against up to KMAX home atoms held wave-uniform.
constexpr int kListCap = 1024;   // candidates a wave lists at a time
constexpr int kCompacted = -2;   // `resident` when the list holds a home group's filtered candidates
constexpr int kFilterSteps = 4;  // candidate steps the filter loads at once
static_assert(kListCap / 64 <= 32, "the list build keeps one bit per 64-candidate step");
constexpr int kMaxStencil = (2 * kTileMaxR + 1) * (2 * kTileMaxR + 1) * (2 * kTileMaxR + 1);
static_assert(kMaxStencil <= 128, "stencil code must fit 7 bits");

template <typename Q>
struct Shift {
  Q x, y, z;   // stencil offset (ox, oy, oz) times the cell edge, in the payload's units
};

// Box b's stencil shift table (kShiftSlots entries, built on the host) into LDS.
template <typename Q>
__device__ __forceinline__ void load_shifts(const Views& v, int b, Shift<Q>* shifts) {
  const Shift<Q>* __restrict__ tab = static_cast<const Shift<Q>*>(v.shift_tab) + (int64_t)b * kShiftSlots;
  static_assert(kShiftSlots == 128, "two entries per lane of one wave");
  if (blockDim.x == 64) {   // one wave: two entries per lane, both loads in flight together
    const Shift<Q> a = tab[threadIdx.x], c = tab[threadIdx.x + 64];
    shifts[threadIdx.x] = a;
    shifts[threadIdx.x + 64] = c;
  } else {
    for (int c = (int)threadIdx.x; c < kShiftSlots; c += (int)blockDim.x) shifts[c] = tab[c];
  }
}

// Exclusive prefix sum of x >= 0 over the wave, bit plane by bit plane: the lanes below
// this one whose bit b is set add 2^b each (a ballot and a masked popcount per plane).
__device__ __forceinline__ int wave_exclusive_scan(int x, int& total) {
  int below = 0, tot = 0;
  for (int b = 0; b < 31; ++b) {
    if (__builtin_amdgcn_ballot_w64((x >> b) != 0) == 0) break;
    const uint64_t m = __builtin_amdgcn_ballot_w64(((x >> b) & 1) != 0);
    below += lanes_below(m) << b;
    tot += __popcll(m) << b;
  }
  total = tot;
  return below;
}

// Writes entries [c0, c0 + kListCap) of home cell lc's candidate list to list[]; returns
// the list's full length (the same on every lane).  Lane l lists stencil codes 2l and
// 2l + 1 (x-neighbours, so consecutive entries are mostly consecutive in memory).
__device__ __forceinline__ int fill_list(const Views& v, const BoxDev& B, int lc, int c0, uint32_t* list) {
  const int ln = lane();
  const int R = v.R, W = 2 * R + 1, W3 = W * W * W;
  const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
  const Cell3 k3 = cell_coords(lc, B);
  // both cells' bounds are loaded together (a code past the stencil reads the home cell's
  // and counts nothing)
  int start[2], n[2], c[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int code = min(2 * ln + h, W3 - 1);
    const Cell3 o = stencil_offset(code, R);
    int nx = k3.x + o.x, ny = k3.y + o.y, nz = k3.z + o.z;
    nx += nx < 0 ? M0 : 0;
    nx -= nx >= M0 ? M0 : 0;
    ny += ny < 0 ? M1 : 0;
    ny -= ny >= M1 ? M1 : 0;
    nz += nz < 0 ? M2 : 0;
    nz -= nz >= M2 ? M2 : 0;
    c[h] = B.cell_off + nx + M0 * (ny + M1 * nz);
  }
  int e[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    start[h] = v.cell_start[c[h]];
    e[h] = v.cell_start[c[h] + 1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) n[h] = 2 * ln + h < W3 ? e[h] - start[h] : 0;
  int total;
  int f = wave_exclusive_scan(n[0] + n[1], total);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int a1 = min(n[h], c0 + kListCap - f);
    for (int a = max(0, c0 - f); a < a1; ++a) list[f + a - c0] = ((uint32_t)(start[h] + a) << 7) | (2 * ln + h);
    f += n[h];
  }
  return total;
}

// The candidate list of home cell lc, entries [c0, c0 + kListCap), into list[]; returns its
// full length.  Cell path: the whole stencil, listed here.  Neighbour-list mode with cell
// lists (LIST): the cell's own list, the candidates within rc + skin of any of its atoms at
// the last build (k_nl_build_tile), copied from HBM; a cell whose list outgrew its capacity
// streams its whole stencil instead (the bins of the build: every atom has moved less than
// half the skin since, and the stencil covers rc + skin, so every pair within rc is in it).
// The chunk is padded with the sentinel entry from its end up to and including the next
// multiple of 64 (list holds kListCap + 65 entries).
template <bool LIST>
__device__ __forceinline__ int load_list(const Views& v, const BoxDev& B, int lc, int c0, uint32_t* list) {
  int n;
  if constexpr (!LIST) {
    n = fill_list(v, B, lc, c0, list);
  } else {
    n = v.nl_count[B.cell_off + lc];
    if (n > v.nl_cap) {
      n = fill_list(v, B, lc, c0, list);
    } else {
      const uint32_t* __restrict__ src = v.nl_list + B.nl_off + (int64_t)lc * v.nl_cap;
      const int m = min(kListCap, n - c0);
      for (int t = lane(); t < m; t += 64) list[t] = src[c0 + t];
    }
  }
  const int cn = min(kListCap, n - c0);
  if (lane() <= ((cn + 63) & ~63) - cn) list[cn + lane()] = kSentinelEntry;
  return n;
}

struct BandEnergy {
  double e, es, w;
};

// Settles the cutoff-band pairs and the close contacts of one home group of a mixed tile wave,
// after its home forces are stored.  The recorded candidate steps (flat list positions) are
// revisited and their band pairs and close contacts queued in (step, home, lane) order,
// refilling the list where a step lies in another chunk.  Each queued band pair is re-decided
// in FP64 and, when outside, its FP32 force is taken back out; each close contact is evaluated
// in FP64 and added.  Both are summed per home over the lanes in a fixed order and applied in
// one rounding by the lane that stored that home (lane k << SHIFT for home k).  With more
// steps or pairs than the slots hold (not expected in a melt) every candidate of the group is
// walked again instead, from the full list (total entries).  LDS executes a wave's accesses in
// order and only this wave wrote its slots, so no barrier is needed.  `resident` is the chunk
// the list holds, or kCompacted when it holds the group's ncand filtered candidates (the
// positions the steps were recorded at); it is updated.
template <bool ENERGY, bool UNI, bool LIST, int SHIFT>
__device__ __forceinline__ BandEnergy settle_group(const Views& v, int chain_len, int excl, double rc2,
                                                   const LjPair<float>& cf, const LjPair<double>& cd,
                                                   const BoxDev& B, Band bd, int lc, int total, int ncand,
                                                   uint32_t* list, int& resident, const Shift<int>* shifts,
                                                   const int* steps, int32_t* bq, const int4* __restrict__ pay,
                                                   int hs, int g0, int kc, int nsteps) {
  const int ln = lane();
  float* f = static_cast<float*>(v.f_lj);
  double e = 0.0, es = 0.0, w = 0.0;
  auto candidate = [&](int t, int cn, int& jx, int& jy, int& jz, int32_t& jt) -> bool {
    jx = jy = jz = 0;
    jt = 0;
    if (t < cn) {
      const uint32_t ent = list[t];
      const int4 q = pay[ent >> 7];
      const Shift<int> sh = shifts[ent & 127];
      jt = pay_tag(q);
      jx = q.x + sh.x;
      jy = q.y + sh.y;
      jz = q.z + sh.z;
    }
    return t < cn;
  };
  auto window = [&](int i, int32_t& hlo, uint32_t& hspan) {
    const int32_t c0 = i - i % chain_len;
    hlo = max(i - excl, c0);
    hspan = (uint32_t)(min(i + excl, c0 + chain_len - 1) - hlo);
  };
  // one queued pair's correction on this lane: band (FP32, units of 2^25) or close (FP64)
  auto correct = [&](int32_t i, int32_t j, int tt, bool close, float& bx, float& by, float& bz, double& cx,
                     double& cy, double& cz) {
    double d[3], r2;
    const bool inside = inside_cutoff_f64(v.pos, v.N, B, i, j, rc2, d, r2);
    if (close)
      add_close_pair<ENERGY>(d, r2, pick(cd.f12, tt), pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt),
                             pick(cd.ecut, tt), cx, cy, cz, e, es, w);
    else if (!inside)
      remove_band_pair<ENERGY>(d, r2, pick(cf.f12, tt), pick(cf.f6, tt), pick(cf.e12, tt), pick(cf.e6, tt),
                               pick(cf.ecut, tt), bx, by, bz, e, es, w);
  };
  // home k's corrections summed over the lanes, added to its stored force in one rounding
  auto apply = [&](int k, float bx, float by, float bz, double cx, double cy, double cz) {
    bx = group_sum(bx, 0);
    by = group_sum(by, 0);
    bz = group_sum(bz, 0);
    cx = group_sum(cx, 0);
    cy = group_sum(cy, 0);
    cz = group_sum(cz, 0);
    if (ln == k << SHIFT) {
      const int32_t i = tag_index(pay_tag(pay[hs + g0 + k]));
      f[i] = (float)((double)f[i] + ((double)(bx * kInvFixF) + cx));
      f[v.N + i] = (float)((double)f[v.N + i] + ((double)(by * kInvFixF) + cy));
      f[2 * v.N + i] = (float)((double)f[2 * v.N + i] + ((double)(bz * kInvFixF) + cz));
    }
  };
  int qn = 0;   // queued pairs: j << 6 | type_j << 5 | close << 4 | k
  if (nsteps <= kBandSteps) {
    for (int s = 0; s < nsteps; ++s) {
      const int fs = steps[s];
      const int c0 = fs - fs % kListCap;
      if (resident != kCompacted && c0 != resident) {
        load_list<LIST>(v, B, lc, c0, list);
        resident = c0;
      }
      int jx, jy, jz;
      int32_t jt;
      const bool act = candidate(fs - c0 + ln, min(kListCap, ncand - c0), jx, jy, jz, jt);
      for (int k = 0; k < kc; ++k) {
        const int4 hq = pay[hs + g0 + k];
        int32_t hlo;
        uint32_t hspan;
        window(tag_index(pay_tag(hq)), hlo, hspan);
        const bool keep = act && (uint32_t)(tag_index(jt) - hlo) > hspan;
        const float r2s = r2_fix((float)(hq.x - jx), (float)(hq.y - jy), (float)(hq.z - jz));
        const bool qc = is_close(r2s, keep, bd);
        const bool qb = qc || in_band(r2s, keep, bd);
        const uint64_t qm = __builtin_amdgcn_ballot_w64(qb);
        const int at = qn + lanes_below(qm);
        if (qb && at < kBandQueue) bq[at] = (tag_index(jt) << 6) | (tag_type(jt) << 5) | ((int)qc << 4) | k;
        qn += __popcll(qm);
      }
    }
  }
  if (nsteps <= kBandSteps && qn <= kBandQueue) {
    float bx = 0.0f, by = 0.0f, bz = 0.0f;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    int kq = -1;
    if (ln < qn) {
      const int32_t ent = bq[ln];
      kq = ent & 15;
      const int32_t htag = pay_tag(pay[hs + g0 + kq]);
      const int tt = UNI ? 0 : tag_type(htag) * 2 + ((ent >> 5) & 1);
      correct(tag_index(htag), ent >> 6, tt, ((ent >> 4) & 1) != 0, bx, by, bz, cx, cy, cz);
    }
    for (int k = 0; k < kc; ++k) {
      if (__builtin_amdgcn_ballot_w64(kq == k) == 0) continue;
      const bool mine = kq == k;
      apply(k, mine ? bx : 0.0f, mine ? by : 0.0f, mine ? bz : 0.0f, mine ? cx : 0.0, mine ? cy : 0.0,
            mine ? cz : 0.0);
    }
  } else {
    for (int k = 0; k < kc; ++k) {
      const int4 hq = pay[hs + g0 + k];
      const int32_t i = tag_index(pay_tag(hq));
      int32_t hlo;
      uint32_t hspan;
      window(i, hlo, hspan);
      float bx = 0.0f, by = 0.0f, bz = 0.0f;
      double cx = 0.0, cy = 0.0, cz = 0.0;
      for (int c0 = 0; c0 < total; c0 += kListCap) {
        if (c0 != resident) {
          load_list<LIST>(v, B, lc, c0, list);
          resident = c0;
        }
        const int cn = min(kListCap, total - c0);
        for (int t0 = 0; t0 < cn; t0 += 64) {
          int jx, jy, jz;
          int32_t jt;
          const bool act = candidate(t0 + ln, cn, jx, jy, jz, jt);
          const int32_t jidx = tag_index(jt);
          const bool keep = act && (uint32_t)(jidx - hlo) > hspan;
          const float r2s = r2_fix((float)(hq.x - jx), (float)(hq.y - jy), (float)(hq.z - jz));
          const bool qc = is_close(r2s, keep, bd);
          if (qc || in_band(r2s, keep, bd))
            correct(i, jidx, UNI ? 0 : tag_type(pay_tag(hq)) * 2 + tag_type(jt), qc, bx, by, bz, cx, cy, cz);
        }
      }
      apply(k, bx, by, bz, cx, cy, cz);
    }
  }
  return BandEnergy{e, es, w};
}

// Sums KMAX per-lane force accumulators (three components each) over the 64 lanes in a
// fixed order.  Recursive halving: at each of the first log2(KMAX) levels a lane keeps half of
// its values and adds the partner's copy of that half, so the 3 KMAX sums take 3 KMAX - 3
// exchanges (instead of 18 KMAX for separate butterflies); then a butterfly over the remaining
// lane bits.  Level lv splits the lanes by bit 5 - lv and exchanges through kLevel[lv] (for
// bit 2 the partner l ^ 7 also differs in bit 2 only among the bits not yet summed).
// Afterwards every lane of [h * 64/KMAX, (h + 1) * 64/KMAX) holds accumulator h's sums.
template <typename P, int KMAX>
__device__ __forceinline__ void sum_homes(int ln, P (&ax)[KMAX], P (&ay)[KMAX], P (&az)[KMAX], P& sx, P& sy,
                                          P& sz) {
  constexpr int LV = KMAX == 16 ? 4 : (KMAX == 8 ? 3 : (KMAX == 4 ? 2 : (KMAX == 2 ? 1 : 0)));
  static_assert((1 << LV) == KMAX, "KMAX must be 1, 2, 4, 8 or 16");
  constexpr int NV = 3 * KMAX;
  P val[NV];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    val[3 * k] = ax[k];
    val[3 * k + 1] = ay[k];
    val[3 * k + 2] = az[k];
  }
#pragma unroll
  for (int lv = 0; lv < LV; ++lv) {
#pragma unroll
    for (int i = 0; i < (NV >> lv) / 2; ++i) {
      const int h = (NV >> lv) / 2 + i;
      if (lv < 2) {
        // lanes below the split keep val[i], those above val[h]
        val[i] = swap_sum(val[i], val[h], kLevel[lv]);
      } else {
        const bool hi = (ln & (32 >> lv)) != 0;
        const P send = hi ? val[i] : val[h];
        const P keep = hi ? val[h] : val[i];
        val[i] = keep + partner(send, lv == 2 ? Xl::Ror8 : Xl::Mirror8);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) val[c] = group_sum(val[c], LV);
  sx = val[0];
  sy = val[1];
  sz = val[2];
}

// Occupancy targets (measured): the mixed form with 8 homes is held to 6 waves per SIMD (80
// VGPRs; it uses 73, with no vector spills), 4 homes to 8 and 16 homes to 4; the FP64 form
// (K = 4) fits 8.
// LIST: neighbour-list mode with per-cell lists (the homes and the sorted order are those of
// the last build, the payload the one refreshed since).
template <bool FP64, bool ENERGY, bool UNI, int KMAX, bool BRANCHLESS, bool LIST = false>
__global__ __launch_bounds__(64 * kTileWaves)
__attribute__((amdgpu_waves_per_eu(FP64 ? 8 : (KMAX >= 16 ? 4 : (KMAX <= 4 ? 8 : 6)))))
void k_lj_tile(Views v, FFDev ff, LjPair<float> cf, LjPair<double> cd) {
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using P = std::conditional_t<FP64, double, float>;
  using Q = std::conditional_t<FP64, double, int>;     // coordinate type
  constexpr int LV = KMAX == 16 ? 4 : (KMAX == 8 ? 3 : (KMAX == 4 ? 2 : (KMAX == 2 ? 1 : 0)));   // log2(KMAX)
  static_assert((1 << LV) == KMAX, "KMAX must be 1, 2, 4, 8 or 16");
  __shared__ uint32_t list[kTileWaves][kListCap + 65];   // + the padding to a whole step, + 1
  __shared__ Shift<Q> shifts[kShiftSlots];
  __shared__ dd red[kTileWaves][3];
  __shared__ int32_t bq[kTileWaves][kBandQueue];   // queued pairs: j << 6 | type_j << 5 | close << 4 | k
  __shared__ int bsteps[kTileWaves][kBandSteps];    // flat list position of each recorded step

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ln = lane();
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
  // home cells (a slab of the box) so its L2 holds one neighbourhood of the payload.
  const int per_xcd = (int)gridDim.x / kXcds;
  const int blk = ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
  if (blk >= v.n_lj_blocks) return;
  const int b = v.lj_blk_box[blk];
  const BoxDev& B = v.boxes[b];
  const int lc = (blk - B.lj_blk_off) * kTileWaves + wave;   // home cell within the box
  const bool wact = lc < B.n_cells;
  const int32_t* __restrict__ cs = v.cell_start;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);

  // stencil offsets in the payload's units (the same for every wave of the block)
  load_shifts(v, b, shifts);
  int total = 0, resident = 0;
  if (wact) total = __builtin_amdgcn_readfirstlane(load_list<LIST>(v, B, lc, 0, list[wave]));
  __syncthreads();

  double e = 0.0, es = 0.0, w = 0.0;
  if (wact) {
    const int hs = __builtin_amdgcn_readfirstlane(cs[B.cell_off + lc]);
    const int hn = __builtin_amdgcn_readfirstlane(cs[B.cell_off + lc + 1]) - hs;
    const Band bd = band_of(cf);
    // one type pair (mixed): forces are summed divided by f6 (see pair_fix)
    const float f12_fold = cf.f12_fold;
    const float fscale = UNI ? kInvFixF * cf.f6[0] : kInvFixF;
    for (int g0 = 0; g0 < hn; g0 += KMAX) {
      const int kc = min(KMAX, hn - g0);
      // The group's homes, one per lane (lane k < kc holds home k), loaded together, with each
      // home's exclusion window (the sorted indices within excl bonds along its chain); then
      // broadcast to wave-uniform values.  A lane past the group holds zeros and a window
      // that excludes every candidate.
      PayT qh{};
      int32_t lo_l = 0, ht_l = 0;
      uint32_t span_l = 0xffffffffu;
      if (ln < kc) {
        qh = pay[hs + g0 + ln];
        const int32_t i = tag_index(pay_tag(qh));
        const int32_t c0 = chain_first(i, ff);
        lo_l = max(i - ff.excl, c0);
        span_l = (uint32_t)(min(i + ff.excl, c0 + ff.chain_len - 1) - lo_l);
        ht_l = tag_type(pay_tag(qh));
      }
      // Cell path with a one-chunk list: keep only the candidates within the cutoff of the
      // box bounding the group's homes (about half of the stencil's atoms in a melt),
      // compacted in place.  Per axis |x - clamp(x, lo, hi)| <= |x - x_home| for every home
      // in the box, and each rounding is monotone, so the filter's r^2 (the pair test's
      // own operation order in the mixed form) never exceeds a pair's: no counted pair is
      // dropped.  Each batch's reads precede its writes and land at or above them.
      int ncand = total;    // list entries the step loop walks
      if (!LIST && total <= kListCap) {
        if (resident != 0) {
          load_list<LIST>(v, B, lc, 0, list[wave]);
          resident = 0;
        }
        // the box bounding the homes, reduced over the first KMAX lanes (in vector registers:
        // the clamp reads both bounds of an axis)
        const bool hv = ln < kc;
        Q lox = first_lanes_min<KMAX>(hv ? qh.x : box_top<Q>()), hix = first_lanes_max<KMAX>(hv ? qh.x : -box_top<Q>());
        Q loy = first_lanes_min<KMAX>(hv ? qh.y : box_top<Q>()), hiy = first_lanes_max<KMAX>(hv ? qh.y : -box_top<Q>());
        Q loz = first_lanes_min<KMAX>(hv ? qh.z : box_top<Q>()), hiz = first_lanes_max<KMAX>(hv ? qh.z : -box_top<Q>());
        const double rc2_keep = ff.rc2 * (1.0 + 1e-12);
        int m = 0;
        constexpr int kFilter = FP64 ? 2 : kFilterSteps;
        // NU steps from position t0 (all below the padded end, whose entries past total are the
        // sentinel, which never passes); a batch reads all its entries before it writes any
        auto batch = [&](int t0, auto nu) {
          constexpr int NU = decltype(nu)::value;
          uint32_t ent[NU];
          Q jx[NU], jy[NU], jz[NU];
#pragma unroll
          for (int u = 0; u < NU; ++u) ent[u] = list[wave][t0 + 64 * u + ln];
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const PayT q = pay[ent[u] >> 7];
            const Shift<Q> sh = shifts[ent[u] & 127];
            jx[u] = q.x + sh.x;
            jy[u] = q.y + sh.y;
            jz[u] = q.z + sh.z;
          }
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const Q dx = jx[u] - clamp_box(jx[u], lox, hix), dy = jy[u] - clamp_box(jy[u], loy, hiy),
                    dz = jz[u] - clamp_box(jz[u], loz, hiz);
            bool pass;
            if constexpr (FP64)
              pass = dx * dx + dy * dy + dz * dz < rc2_keep;
            else
              pass = r2_fix((float)dx, (float)dy, (float)dz) < bd.hi;
            const uint64_t bm = __builtin_amdgcn_ballot_w64(pass);
            if (pass) list[wave][m + lanes_below(bm)] = ent[u];
            m += __popcll(bm);
          }
        };
        // whole batches of kFilter steps with their loads in flight together, then single steps
        const int tp = (total + 63) & ~63;
        int t0 = 0;
        for (; t0 + 64 * kFilter <= tp; t0 += 64 * kFilter) batch(t0, std::integral_constant<int, kFilter>());
        for (; t0 < tp; t0 += 64) batch(t0, std::integral_constant<int, 1>());
        if (ln < ((m + 63) & ~63) - m) list[wave][m + ln] = kSentinelEntry;   // pad to whole steps
        ncand = m;
        resident = kCompacted;
      }
      // the homes broadcast to wave-uniform values (after the filter, which needs only their box)
      Q hx[KMAX], hy[KMAX], hz[KMAX];
      int32_t lo[KMAX], hti[KMAX];
      uint32_t span[KMAX];
      P ax[KMAX], ay[KMAX], az[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        ax[k] = ay[k] = az[k] = (P)0;
        hx[k] = lane_value(qh.x, k);
        hy[k] = lane_value(qh.y, k);
        hz[k] = lane_value(qh.z, k);
        lo[k] = lane_value(lo_l, k);
        span[k] = (uint32_t)lane_value((int32_t)span_l, k);
        hti[k] = lane_value(ht_l, k);
      }
      int nsteps = 0;       // candidate steps with a band pair or a close contact (wave-uniform)
      int32_t bmax = 0;     // bits of the largest r2s counted since the last band check
      for (int c0 = 0; c0 < ncand; c0 += kListCap) {
        if (resident != kCompacted && c0 != resident) {
          load_list<LIST>(v, B, lc, c0, list[wave]);
          resident = c0;
        }
        const int cn = min(kListCap, ncand - c0);
        for (int t0 = 0; t0 < cn; t0 += 64) {
          // the list is padded to whole steps with the sentinel, which lies beyond the cutoff
          const uint32_t ent = list[wave][t0 + ln];
          const PayT q = pay[ent >> 7];
          const Shift<Q> sh = shifts[ent & 127];
          const int32_t jt = pay_tag(q);
          const Q jx = q.x + sh.x, jy = q.y + sh.y, jz = q.z + sh.z;
          const int32_t jidx = tag_index(jt);
          const int jtype = tag_type(jt);
          bool near = false;    // a close contact on this lane in this step (mixed)
          // the group's home count, re-read each step as an opaque scalar: the compiler then
          // tests k < kc with a scalar compare per home instead of holding KMAX lane masks
          int kcs = kc;
          asm volatile("" : "+s"(kcs));
#pragma unroll
          for (int k = 0; k < KMAX; ++k) {
            if (k < kcs) {
              const bool keep = (uint32_t)(jidx - lo[k]) > span[k];
              const int tt = UNI ? 0 : hti[k] * 2 + jtype;
              if constexpr (FP64)
                pair_f64<ENERGY>(hx[k] - jx, hy[k] - jy, hz[k] - jz, keep, ff.rc2, pick(cd.f12, tt),
                                 pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt), pick(cd.ecut, tt), ax[k],
                                 ay[k], az[k], e, es, w);
              else
                pair_fix<ENERGY, BRANCHLESS, UNI>(hx[k] - jx, hy[k] - jy, hz[k] - jz, keep, bd,
                                                  UNI ? f12_fold : pick(cf.f12, tt), pick(cf.f6, tt),
                                                  pick(cf.e12, tt), pick(cf.e6, tt), pick(cf.ecut, tt), ax[k],
                                                  ay[k], az[k], e, es, w, bmax, near);
            }
          }
          if constexpr (!FP64) {
            // rare: a lane counted a pair in the cutoff band or met a close contact; note the step
            if (__builtin_amdgcn_ballot_w64(bmax >= __float_as_int(bd.lo) || near) != 0) {
              bmax = 0;
              if (nsteps < kBandSteps && ln == 0) bsteps[wave][nsteps] = c0 + t0;
              ++nsteps;
            }
          }
        }
      }
      // Sum each home atom's partial forces over the 64 lanes in a fixed order, as sum_homes
      // does (written out here: the explicit exchange patterns keep the register allocation
      // tighter): lanes [h * 64/KMAX, (h + 1) * 64/KMAX) then hold home h's sums, and the first
      // of them stores it (and later applies its band and close-contact corrections).
      P* f = static_cast<P*>(v.f_lj);
      {
        constexpr int NV = 3 * KMAX;
        P val[NV];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          val[3 * k] = ax[k];
          val[3 * k + 1] = ay[k];
          val[3 * k + 2] = az[k];
        }
#pragma unroll
        for (int lv = 0; lv < LV; ++lv) {
#pragma unroll
          for (int i = 0; i < (NV >> lv) / 2; ++i) {
            const int h = (NV >> lv) / 2 + i;
            if (lv < 2) {
              val[i] = swap_sum(val[i], val[h], kLevel[lv]);
            } else {
              const bool hi = (ln & (32 >> lv)) != 0;
              const P send = hi ? val[i] : val[h];
              const P keep = hi ? val[h] : val[i];
              val[i] = keep + partner(send, lv == 2 ? Xl::Ror8 : Xl::Mirror8);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) val[c] = group_sum(val[c], LV);
        P sx = val[0], sy = val[1], sz = val[2];
        if constexpr (!FP64) {
          sx *= fscale;
          sy *= fscale;
          sz *= fscale;
        }
        const int hk = ln >> (6 - LV);
        const int32_t i = tag_index(__shfl(pay_tag(qh), hk));   // home hk's index, from lane hk
        if ((ln & ((64 >> LV) - 1)) == 0 && hk < kc) {
          f[i] = sx;
          f[v.N + i] = sy;
          f[2 * v.N + i] = sz;
        }
      }
      if constexpr (!FP64) {
        if (nsteps > 0) {
          const BandEnergy be = settle_group<ENERGY, UNI, LIST, 6 - LV>(v, ff.chain_len, ff.excl, ff.rc2, cf, cd, B, bd,
                                                                       lc, total, ncand, list[wave], resident, shifts,
                                                                       bsteps[wave], bq[wave], pay, hs, g0, kc, nsteps);
          if (ENERGY) {
            e += be.e;
            es += be.es;
            w += be.w;
          }
        }
      }
    }
  }
  if (ENERGY) block_energy<kTileWaves>(e, es, w, red, v.part_lj + (int64_t)blk * 3);
}

// ---------------------------------------------------------------------------------
// Newton-3 half shell (MD_LJ_HALFSHELL, opt-in; Section 4.2 names as a cost of its
// thread-per-atom kernels that every pair is computed twice).  Each pair is evaluated once:
// a home cell's wave lists its own atoms and the forward half of its stencil (codes above the
// centre), and takes an in-cell pair only from the lower of the two sorted positions.  The
// force on each candidate (the reaction, summed on its lane over the group's homes) and on
// each home (summed over the lanes) are added to per-atom int64 fixed-point accumulators
// (units of 2^-32 kcal/mol/A) with device atomics.  Integer sums do not depend on the order of
// the additions, so the result is deterministic; k_half_finish turns the accumulators into the
// force array and clears them for the next evaluation.  Band pairs are decided from the FP64
// positions before they are counted.
constexpr double kHalfFix = 4294967296.0;   // accumulator units per kcal/mol/A

// List of home cell lc for the half shell, entries [c0, c0 + kListCap): lane 0 lists the home
// cell (its atoms come first, at positions [0, hn)), lanes 1..(W^3 - 1)/2 the forward cells.
__device__ __forceinline__ int fill_list_half(const Views& v, const BoxDev& B, int lc, int c0, uint32_t* list) {
  const int ln = lane();
  const int R = v.R, W = 2 * R + 1, W3 = W * W * W, ctr = (W3 - 1) / 2;
  const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
  const Cell3 k3 = cell_coords(lc, B);
  const int code = ctr + ln;
  int start = 0, n = 0;
  if (code < W3) {
    const Cell3 o = stencil_offset(code, R);
    int nx = k3.x + o.x, ny = k3.y + o.y, nz = k3.z + o.z;
    nx += nx < 0 ? M0 : 0;
    nx -= nx >= M0 ? M0 : 0;
    ny += ny < 0 ? M1 : 0;
    ny -= ny >= M1 ? M1 : 0;
    nz += nz < 0 ? M2 : 0;
    nz -= nz >= M2 ? M2 : 0;
    const int c = B.cell_off + nx + M0 * (ny + M1 * nz);
    start = v.cell_start[c];
    n = v.cell_start[c + 1] - start;
  }
  int total;
  const int f = wave_exclusive_scan(n, total);
  const int a1 = min(n, c0 + kListCap - f);
  for (int a = max(0, c0 - f); a < a1; ++a) list[f + a - c0] = ((uint32_t)(start + a) << 7) | code;
  return total;
}

// Adds x (in units of 1/scale kcal/mol/A) to an int64 fixed-point accumulator.
__device__ __forceinline__ void deposit(unsigned long long* a, double x) {
  atomicAdd(a, (unsigned long long)__double2ll_rn(x));
}

template <bool FP64, bool ENERGY>
__global__ __launch_bounds__(64 * kTileWaves) void k_lj_half(Views v, FFDev ff, LjPair<float> cf, LjPair<double> cd) {
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using P = std::conditional_t<FP64, double, float>;
  using Q = std::conditional_t<FP64, double, int>;
  constexpr int KMAX = FP64 ? 4 : 8;
  constexpr int LV = FP64 ? 2 : 3;
  __shared__ uint32_t list[kTileWaves][kListCap];
  __shared__ Shift<Q> shifts[kShiftSlots];
  __shared__ dd red[kTileWaves][3];

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ln = lane();
  const int per_xcd = (int)gridDim.x / kXcds;
  const int blk = ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
  if (blk >= v.n_lj_blocks) return;
  const BoxDev& B = v.boxes[v.lj_blk_box[blk]];
  const int lc = (blk - B.lj_blk_off) * kTileWaves + wave;
  const bool wact = lc < B.n_cells;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);
  const int R = v.R, W = 2 * R + 1, ctr = (W * W * W - 1) / 2;
  load_shifts(v, v.lj_blk_box[blk], shifts);
  int total = 0, resident = 0;
  if (wact) total = __builtin_amdgcn_readfirstlane(fill_list_half(v, B, lc, 0, list[wave]));
  __syncthreads();

  double e = 0.0, es = 0.0, w = 0.0;
  if (wact) {
    const int hs = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc]);
    const int hn = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc + 1]) - hs;
    const Band bd = band_of(cf);
    // accumulator units per unit of the lane sums: mixed sums are in 2^25 (fixed-point) units
    const double scale = FP64 ? kHalfFix : kHalfFix * (double)kInvFixF;
    unsigned long long* __restrict__ acc = v.f_acc;
    const int64_t N = v.N;
    for (int g0 = 0; g0 < hn; g0 += KMAX) {
      const int kc = min(KMAX, hn - g0);
      Q hx[KMAX], hy[KMAX], hz[KMAX];
      int32_t lo[KMAX], hti[KMAX], hidx[KMAX];
      uint32_t span[KMAX];
      P ax[KMAX], ay[KMAX], az[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        ax[k] = ay[k] = az[k] = (P)0;
        hx[k] = hy[k] = hz[k] = (Q)0;
        lo[k] = hti[k] = hidx[k] = 0;
        span[k] = 0xffffffffu;   // excludes every candidate
        if (k < kc) {
          const PayT q = pay[hs + g0 + k];
          hx[k] = q.x;
          hy[k] = q.y;
          hz[k] = q.z;
          const int32_t tag = pay_tag(q);
          const int32_t i = tag_index(tag);
          const int32_t c0 = chain_first(i, ff);
          hidx[k] = i;
          lo[k] = max(i - ff.excl, c0);
          span[k] = (uint32_t)(min(i + ff.excl, c0 + ff.chain_len - 1) - lo[k]);
          hti[k] = tag_type(tag);
        }
      }
      for (int c0 = 0; c0 < total; c0 += kListCap) {
        if (c0 != resident) {
          fill_list_half(v, B, lc, c0, list[wave]);
          resident = c0;
        }
        const int cn = min(kListCap, total - c0);
        for (int t0 = 0; t0 < cn; t0 += 64) {
          const bool act = t0 + ln < cn;
          Q jx = (Q)0, jy = (Q)0, jz = (Q)0;
          int32_t jt = 0;
          uint32_t ent = 0;
          if (act) {
            ent = list[wave][t0 + ln];
            const PayT q = pay[ent >> 7];
            const Shift<Q> sh = shifts[ent & 127];
            jt = pay_tag(q);
            jx = q.x + sh.x;
            jy = q.y + sh.y;
            jz = q.z + sh.z;
          }
          const int32_t jidx = tag_index(jt);
          const int jtype = tag_type(jt);
          // in-cell candidates (list positions [0, hn)) pair only with homes at lower positions
          const bool own_cell = c0 + t0 < hn;
          const int jpos = (int)(ent >> 7);
          P cx = (P)0, cy = (P)0, cz = (P)0;   // force on the candidate
#pragma unroll
          for (int k = 0; k < KMAX; ++k) {
            if (k < kc) {
              bool keep = act && (uint32_t)(jidx - lo[k]) > span[k];
              if (own_cell) keep = keep && ((int)(ent & 127) != ctr || jpos > hs + g0 + k);
              const int tt = ff.uniform_lj ? 0 : hti[k] * 2 + jtype;
              if constexpr (FP64) {
                const double dx = hx[k] - jx, dy = hy[k] - jy, dz = hz[k] - jz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (keep && r2 < ff.rc2) {
                  const double r2i = 1.0 / r2;
                  const double r6 = r2i * r2i * r2i;
                  const double g = r6 * (pick(cd.f12, tt) * r6 - pick(cd.f6, tt));
                  const double ffs = g * r2i;
                  ax[k] += ffs * dx;
                  ay[k] += ffs * dy;
                  az[k] += ffs * dz;
                  cx -= ffs * dx;
                  cy -= ffs * dy;
                  cz -= ffs * dz;
                  if (ENERGY) {
                    const double en = r6 * (pick(cd.e12, tt) * r6 - pick(cd.e6, tt));
                    e += en;
                    es += en - pick(cd.ecut, tt);
                    w += g;
                  }
                }
              } else {
                const float dx = (float)(hx[k] - jx), dy = (float)(hy[k] - jy), dz = (float)(hz[k] - jz);
                const float r2s = r2_fix(dx, dy, dz);
                bool hit = keep && r2s < bd.hi;
                if (hit && r2s >= bd.lo) {
                  // rare: FP32 cannot tell the side of the cutoff; decide from the FP64 positions
                  double d[3], r2;
                  hit = inside_cutoff_f64(v.pos, N, B, hidx[k], jidx, ff.rc2, d, r2);
                }
                if (is_close(r2s, keep, bd)) {
                  // rare: a close contact, evaluated in FP64 and deposited on both atoms at once
                  double d[3], r2, fx = 0.0, fy = 0.0, fz = 0.0;
                  inside_cutoff_f64(v.pos, N, B, hidx[k], jidx, ff.rc2, d, r2);
                  add_close_pair<ENERGY>(d, r2, pick(cd.f12, tt), pick(cd.f6, tt), pick(cd.e12, tt),
                                         pick(cd.e6, tt), pick(cd.ecut, tt), fx, fy, fz, e, es, w);
                  deposit(acc + hidx[k], fx * kHalfFix);
                  deposit(acc + N + hidx[k], fy * kHalfFix);
                  deposit(acc + 2 * N + hidx[k], fz * kHalfFix);
                  deposit(acc + jidx, -fx * kHalfFix);
                  deposit(acc + N + jidx, -fy * kHalfFix);
                  deposit(acc + 2 * N + jidx, -fz * kHalfFix);
                  hit = false;
                }
                if (hit) {
                  const float r2 = r2s * kInvFix2F;
                  const float r2i = rcp_f(r2);
                  const float r6 = r2i * r2i * r2i;
                  const float g = r6 * (pick(cf.f12, tt) * r6 - pick(cf.f6, tt));
                  const float ffs = g * r2i;
                  ax[k] += ffs * dx;
                  ay[k] += ffs * dy;
                  az[k] += ffs * dz;
                  cx -= ffs * dx;
                  cy -= ffs * dy;
                  cz -= ffs * dz;
                  if (ENERGY) {
                    const float en = r6 * (pick(cf.e12, tt) * r6 - pick(cf.e6, tt));
                    e += (double)en;
                    es += (double)en - (double)pick(cf.ecut, tt);
                    w += (double)g;
                  }
                }
              }
            }
          }
          if (act && (cx != (P)0 || cy != (P)0 || cz != (P)0)) {
            deposit(acc + jidx, (double)cx * scale);
            deposit(acc + N + jidx, (double)cy * scale);
            deposit(acc + 2 * N + jidx, (double)cz * scale);
          }
        }
      }
      P sx, sy, sz;
      sum_homes<P, KMAX>(ln, ax, ay, az, sx, sy, sz);
      const int hk = ln >> (6 - LV);
      if ((ln & ((64 >> LV) - 1)) == 0 && hk < kc) {
        const int32_t i = tag_index(pay_tag(pay[hs + g0 + hk]));
        deposit(acc + i, (double)sx * scale);
        deposit(acc + N + i, (double)sy * scale);
        deposit(acc + 2 * N + i, (double)sz * scale);
      }
    }
  }
  // each pair counted once: the block sums halve, so pass twice the pair sums
  if (ENERGY) block_energy<kTileWaves>(2.0 * e, 2.0 * es, 2.0 * w, red, v.part_lj + (int64_t)blk * 3);
}

// Accumulators -> force array (FP32 or FP64), and back to zero for the next evaluation.
template <typename P>
__global__ __launch_bounds__(256) void k_half_finish(Views v) {
  const int64_t n3 = 3 * v.N;
  P* f = static_cast<P*>(v.f_lj);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n3; e += (int64_t)gridDim.x * 256) {
    const long long a = (long long)v.f_acc[e];
    f[e] = (P)((double)a * (1.0 / kHalfFix));
    v.f_acc[e] = 0ull;
  }
}

// ---------------------------------------------------------------------------------
// Neighbour-list mode (Sections 3.1-3.2: the paper's list, rebuilt every few steps).
//
// Build: one wave per home cell, exactly as the cell tile streams its candidates, but a
// pair closer than rc + skin (and not excluded) appends the candidate's list entry to the
// home atom's list instead of computing a force.  Lists are stored per 64 atoms of
// sorted order, entry-major ([nl_cap][64]), so that the force kernel's 64 lanes read 64
// consecutive words per step.
template <bool FP64, int KMAX>
__global__ __launch_bounds__(64 * kTileWaves) void k_nl_build(Views v, FFDev ff, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;   // no rebuild this step
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using Q = std::conditional_t<FP64, double, int>;
  __shared__ uint32_t list[kTileWaves][kListCap];
  __shared__ Shift<Q> shifts[kShiftSlots];

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ln = lane();
  const int per_xcd = (int)gridDim.x / kXcds;
  const int blk = ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
  if (blk >= v.n_cell_blocks) return;
  const BoxDev& B = v.boxes[v.cell_blk_box[blk]];
  const int lc = (blk - B.cell_blk_off) * kTileWaves + wave;
  const bool wact = lc < B.n_cells;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);
  load_shifts(v, v.cell_blk_box[blk], shifts);
  int total = 0, resident = 0;
  if (wact) total = __builtin_amdgcn_readfirstlane(fill_list(v, B, lc, 0, list[wave]));
  __syncthreads();
  if (!wact) return;
  const int hs = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc]);
  const int hn = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc + 1]) - hs;
  // list radius in the payload's units, widened a little: the list may hold extra pairs,
  // never miss one
  const double rl2 = v.nl_rl2 * (1.0 + 1e-5);
  const float rl2s = (float)(rl2 * kFix * kFix);
  const int cap = v.nl_cap;
  for (int g0 = 0; g0 < hn; g0 += KMAX) {
    const int kc = min(KMAX, hn - g0);
    Q hx[KMAX], hy[KMAX], hz[KMAX];
    int32_t lo[KMAX], cnt[KMAX];
    uint32_t span[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      cnt[k] = 0;
      if (k < kc) {
        const PayT q = pay[hs + g0 + k];
        hx[k] = uni(q.x);
        hy[k] = uni(q.y);
        hz[k] = uni(q.z);
        const int32_t i = tag_index(uni(pay_tag(q)));
        const int32_t c0 = chain_first(i, ff);
        lo[k] = max(i - ff.excl, c0);
        span[k] = (uint32_t)(min(i + ff.excl, c0 + ff.chain_len - 1) - lo[k]);
      } else {
        hx[k] = hy[k] = hz[k] = (Q)0;
        lo[k] = 0;
        span[k] = 0xffffffffu;
      }
    }
    for (int c0 = 0; c0 < total; c0 += kListCap) {
      if (c0 != resident) {
        fill_list(v, B, lc, c0, list[wave]);
        resident = c0;
      }
      const int cn = min(kListCap, total - c0);
      for (int t0 = 0; t0 < cn; t0 += 64) {
        const bool act = t0 + ln < cn;
        uint32_t ent = 0;
        Q jx = (Q)0, jy = (Q)0, jz = (Q)0;
        int32_t jt = 0;
        if (act) {
          ent = list[wave][t0 + ln];
          const PayT q = pay[ent >> 7];
          const Shift<Q> sh = shifts[ent & 127];
          jt = pay_tag(q);
          jx = q.x + sh.x;
          jy = q.y + sh.y;
          jz = q.z + sh.z;
        }
        const int32_t jidx = tag_index(jt);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < kc) {
            bool hit;
            if constexpr (FP64) {
              const double dx = hx[k] - jx, dy = hy[k] - jy, dz = hz[k] - jz;
              hit = dx * dx + dy * dy + dz * dz < rl2;
            } else {
              const float dx = (float)(hx[k] - jx), dy = (float)(hy[k] - jy), dz = (float)(hz[k] - jz);
              hit = r2_fix(dx, dy, dz) < rl2s;
            }
            hit = hit && act && (uint32_t)(jidx - lo[k]) > span[k];
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            const int at = cnt[k] + lanes_below(m);
            if (hit && at < cap) {
              const int ls = hs + g0 + k - B.atom_off;   // box-local sorted slot of the home
              v.nl_list[B.nl_off + (int64_t)(ls >> 6) * 64 * cap + (int64_t)at * 64 + (ls & 63)] = ent;
            }
            cnt[k] += __popcll(m);
          }
        }
      }
    }
    // the full count: above cap the force kernel walks this atom's stencil instead
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < kc && ln == 0) v.nl_count[hs + g0 + k] = cnt[k];
  }
}

// Build with per-cell lists: one wave per home cell streams its stencil as the cell tile
// does and keeps every candidate within rc + skin of ANY atom of the cell (the union of
// their Verlet spheres, in stencil order), so the force kernel can stream it exactly like
// the stencil (k_lj_tile<LIST>): fewer candidates, the same coalesced loads.  Home atoms
// and excluded partners stay in the list (the force kernel tests exclusions per pair).
template <bool FP64>
__global__ __launch_bounds__(64 * kTileWaves) void k_nl_build_tile(Views v, FFDev ff, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;   // no rebuild this step
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using Q = std::conditional_t<FP64, double, int>;
  __shared__ uint32_t list[kTileWaves][kListCap];
  __shared__ Shift<Q> shifts[kShiftSlots];

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ln = lane();
  const int per_xcd = (int)gridDim.x / kXcds;
  const int blk = ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
  if (blk >= v.n_cell_blocks) return;
  const BoxDev& B = v.boxes[v.cell_blk_box[blk]];
  const int lc = (blk - B.cell_blk_off) * kTileWaves + wave;
  const bool wact = lc < B.n_cells;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);
  load_shifts(v, v.cell_blk_box[blk], shifts);
  int total = 0, resident = 0;
  if (wact) total = __builtin_amdgcn_readfirstlane(fill_list(v, B, lc, 0, list[wave]));
  __syncthreads();
  if (!wact) return;
  const int hs = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc]);
  const int hn = __builtin_amdgcn_readfirstlane(v.cell_start[B.cell_off + lc + 1]) - hs;
  // list radius, widened a little: the list may hold extra pairs, never miss one
  const double rl2 = v.nl_rl2 * (1.0 + 1e-5);
  const float rl2s = (float)(rl2 * kFix * kFix);
  const int cap = v.nl_cap;
  uint32_t* __restrict__ out = v.nl_list + B.nl_off + (int64_t)lc * cap;
  constexpr int KB = FP64 ? 4 : 8;   // homes held in registers at a time
  int cnt = 0;
  for (int c0 = 0; c0 < total; c0 += kListCap) {
    if (c0 != resident) {
      fill_list(v, B, lc, c0, list[wave]);
      resident = c0;
    }
    const int cn = min(kListCap, total - c0);
    // bit s: the candidate of step s (list position c0 + 64 s + lane) is within reach of a home
    uint32_t hits = 0;
    for (int g0 = 0; g0 < hn; g0 += KB) {
      const int kc = min(KB, hn - g0);
      Q hx[KB], hy[KB], hz[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        hx[k] = hy[k] = hz[k] = (Q)0;
        if (k < kc) {
          const PayT q = pay[hs + g0 + k];
          hx[k] = q.x;
          hy[k] = q.y;
          hz[k] = q.z;
        }
      }
      for (int t0 = 0, s = 0; t0 < cn; t0 += 64, ++s) {
        if (t0 + ln >= cn) continue;
        const uint32_t ent = list[wave][t0 + ln];
        const PayT q = pay[ent >> 7];
        const Shift<Q> sh = shifts[ent & 127];
        const Q jx = q.x + sh.x, jy = q.y + sh.y, jz = q.z + sh.z;
        bool hit = false;
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (k < kc) {
            if constexpr (FP64) {
              const double dx = hx[k] - jx, dy = hy[k] - jy, dz = hz[k] - jz;
              hit = hit || dx * dx + dy * dy + dz * dz < rl2;
            } else {
              hit = hit || r2_fix((float)(hx[k] - jx), (float)(hy[k] - jy), (float)(hz[k] - jz)) < rl2s;
            }
          }
        }
        if (hit) hits |= 1u << s;
      }
    }
    // compaction in list order
    for (int t0 = 0, s = 0; t0 < cn; t0 += 64, ++s) {
      const bool hit = (hits >> s) & 1u;
      const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
      const int at = cnt + lanes_below(m);
      if (hit && at < cap) out[at] = list[wave][t0 + ln];
      cnt += __popcll(m);
    }
  }
  // the full count: above cap the force kernel streams this cell's stencil instead
  if (ln == 0) v.nl_count[B.cell_off + lc] = cnt;
}

// LJ force from the lists: one lane per atom of sorted order, walking its list; the
// candidate comes from the current payload plus the stencil shift recorded at the
// build.  Mixed form: FP32 on exact int32 differences, with the cutoff band decided in
// FP64 (inline: about one list entry in 10^6).
template <bool FP64, bool ENERGY, bool UNI>
__global__ __launch_bounds__(kLjNlBlock) void k_lj_nl(Views v, FFDev ff, LjPair<float> cf, LjPair<double> cd,
                                                    const void* payv) {
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using P = std::conditional_t<FP64, double, float>;
  using Q = std::conditional_t<FP64, double, int>;
  __shared__ Shift<Q> shifts[kShiftSlots];
  __shared__ dd red[kLjNlBlock / 64][3];
  const BoxDev& B = v.boxes[v.lj_blk_box[blockIdx.x]];
  const int local = ((int)blockIdx.x - B.lj_blk_off) * kLjNlBlock + (int)threadIdx.x;
  load_shifts(v, v.lj_blk_box[blockIdx.x], shifts);
  __syncthreads();
  double e = 0.0, es = 0.0, w = 0.0;
  if (local < B.n_atoms) {
    const PayT* __restrict__ pay = static_cast<const PayT*>(payv);
    const int32_t s = B.atom_off + local;
    const PayT hq = pay[s];
    const int32_t i = tag_index(pay_tag(hq));
    const int ti = tag_type(pay_tag(hq));
    const int n = v.nl_count[s];
    const uint32_t* __restrict__ row =
        v.nl_list + B.nl_off + (int64_t)(local >> 6) * 64 * v.nl_cap + (local & 63);
    const Band bd = band_of(cf);
    const float f12_fold = cf.f12[0] / cf.f6[0];
    // kNlSums interleaved partial sums: shorter FP32 summation chains, and that many list
    // entries in flight per lane
    constexpr int kNlSums = FP64 ? 4 : 8;
    P ax[kNlSums], ay[kNlSums], az[kNlSums];
#pragma unroll
    for (int u = 0; u < kNlSums; ++u) ax[u] = ay[u] = az[u] = (P)0;
    double cx = 0.0, cy = 0.0, cz = 0.0;   // close contacts (mixed), FP64
    int32_t bmax = 0;
    // one candidate (payload q at stencil shift sh) into partial sum u
    auto one = [&](const PayT& q, const Shift<Q>& sh, bool keep, int u) {
      const int32_t tj = pay_tag(q);
      const int tt = UNI ? 0 : ti * 2 + tag_type(tj);
      if constexpr (FP64) {
        pair_f64<ENERGY>(hq.x - (q.x + sh.x), hq.y - (q.y + sh.y), hq.z - (q.z + sh.z), keep, ff.rc2,
                         pick(cd.f12, tt), pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt), pick(cd.ecut, tt),
                         ax[u], ay[u], az[u], e, es, w);
      } else {
        const int dqx = hq.x - (q.x + sh.x), dqy = hq.y - (q.y + sh.y), dqz = hq.z - (q.z + sh.z);
        bool near = false;
        const float r2s = pair_fix<ENERGY, false, UNI>(dqx, dqy, dqz, keep, bd, UNI ? f12_fold : pick(cf.f12, tt),
                                                       pick(cf.f6, tt), pick(cf.e12, tt), pick(cf.e6, tt),
                                                       pick(cf.ecut, tt), ax[u], ay[u], az[u], e, es, w, bmax, near);
        double d[3], r2;
        if (near) {   // rare: a close contact, in FP64
          inside_cutoff_f64(v.pos, v.N, B, i, tag_index(tj), ff.rc2, d, r2);
          add_close_pair<ENERGY>(d, r2, pick(cd.f12, tt), pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt),
                                 pick(cd.ecut, tt), cx, cy, cz, e, es, w);
        }
        if (in_band(r2s, keep, bd) && !inside_cutoff_f64(v.pos, v.N, B, i, tag_index(tj), ff.rc2, d, r2)) {
          // counted above as inside; in the folded form the sums are divided by f6
          float bx = 0.0f, by = 0.0f, bz = 0.0f;
          remove_band_pair<ENERGY>(d, r2, pick(cf.f12, tt), pick(cf.f6, tt), pick(cf.e12, tt), pick(cf.e6, tt),
                                   pick(cf.ecut, tt), bx, by, bz, e, es, w);
          const float sc = UNI ? 1.0f / cf.f6[0] : 1.0f;
          ax[u] += bx * sc;
          ay[u] += by * sc;
          az[u] += bz * sc;
        }
      }
    };
    if (n <= v.nl_cap) {
      for (int t0 = 0; t0 < n; t0 += kNlSums) {
#pragma unroll
        for (int u = 0; u < kNlSums; ++u) {
          const int t = t0 + u;
          if (t < n) {
            const uint32_t ent = row[(int64_t)t * 64];
            one(pay[ent >> 7], shifts[ent & 127], true, u);
          }
        }
      }
    } else {
      // the list outgrew its capacity: walk the stencil of the build's bins (every atom has moved
      // less than half the skin since, and the stencil covers rc + skin), excluding 1-2/1-3 here
      const int32_t c0 = chain_first(i, ff);
      const int32_t lo = max(i - ff.excl, c0);
      const uint32_t span = (uint32_t)(min(i + ff.excl, c0 + ff.chain_len - 1) - lo);
      const int R = v.R, W = 2 * R + 1;
      const Cell3 k3 = cell_coords(v.scell[s] - B.cell_off, B);
      for (int code = 0; code < W * W * W; ++code) {
        const Cell3 o = stencil_offset(code, R);
        int nx = k3.x + o.x, ny = k3.y + o.y, nz = k3.z + o.z;
        nx += nx < 0 ? B.M[0] : 0;
        nx -= nx >= B.M[0] ? B.M[0] : 0;
        ny += ny < 0 ? B.M[1] : 0;
        ny -= ny >= B.M[1] ? B.M[1] : 0;
        nz += nz < 0 ? B.M[2] : 0;
        nz -= nz >= B.M[2] ? B.M[2] : 0;
        const int c = B.cell_off + nx + B.M[0] * (ny + B.M[1] * nz);
        for (int t = v.cell_start[c]; t < v.cell_start[c + 1]; ++t) {
          const PayT q = pay[t];
          one(q, shifts[code], (uint32_t)(tag_index(pay_tag(q)) - lo) > span, 0);
        }
      }
    }
    for (int h = kNlSums / 2; h > 0; h >>= 1)   // pairwise
#pragma unroll
      for (int u = 0; u < h; ++u) {
        ax[u] += ax[u + h];
        ay[u] += ay[u + h];
        az[u] += az[u + h];
      }
    P fx = ax[0], fy = ay[0], fz = az[0];
    if constexpr (!FP64) {
      const float sc = UNI ? kInvFixF * cf.f6[0] : kInvFixF;
      fx = (float)((double)(fx * sc) + cx);
      fy = (float)((double)(fy * sc) + cy);
      fz = (float)((double)(fz * sc) + cz);
    }
    P* f = static_cast<P*>(v.f_lj);
    f[i] = fx;
    f[v.N + i] = fy;
    f[2 * v.N + i] = fz;
  }
  if (ENERGY) block_energy<kLjNlBlock / 64>(e, es, w, red, v.part_lj + (int64_t)blockIdx.x * 3);
}

template <typename P>
LjPair<P> make_pair(const FFDev& ff) {
  LjPair<P> c;
  for (int t = 0; t < 4; ++t) {
    c.f12[t] = (P)ff.f12[t];
    c.f6[t] = (P)ff.f6[t];
    c.e12[t] = (P)ff.e12[t];
    c.e6[t] = (P)ff.e6[t];
    c.ecut[t] = (P)ff.ecut[t];
  }
  c.f12_fold = c.f12[0] / c.f6[0];
  c.band_lo = (float)(ff.rc2 * kFix * kFix * (1.0 - kBand));
  c.band_hi = (float)(ff.rc2 * kFix * kFix * (1.0 + kBand));
  // close contacts: r below kCloseSigma times the smallest sigma of a type pair that interacts
  // (sigma^6 = e12 / e6)
  double s6 = 0.0;
  for (int t = 0; t < 4; ++t)
    if (ff.e6[t] > 0.0) s6 = s6 > 0.0 ? std::min(s6, ff.e12[t] / ff.e6[t]) : ff.e12[t] / ff.e6[t];
  c.close = (float)(kCloseSigma * kCloseSigma * std::cbrt(s6) * kFix * kFix);
  return c;
}

template <bool FP64, bool ENERGY, int K, bool LIST>
void launch_tile_k(const Views& v, const FFDev& ff, const LjPair<float>& cf, const LjPair<double>& cd,
                   bool branchless, hipStream_t s) {
  dim3 g((v.n_lj_blocks + kXcds - 1) / kXcds * kXcds), b(64 * kTileWaves);
  if (ff.uniform_lj) {
    if (branchless && !LIST)
      hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, true, K, true>), g, b, 0, s, v, ff, cf, cd);
    else
      hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, true, K, false, LIST>), g, b, 0, s, v, ff, cf, cd);
  } else {
    hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, false, K, false, LIST>), g, b, 0, s, v, ff, cf, cd);
  }
}

// homes: home atoms per pass of a wave (4, 8 or 16; the FP64 form holds 4 in scalar registers).
template <bool FP64, bool ENERGY, bool LIST = false>
void launch_tile(const Views& v, const FFDev& ff, const LjPair<float>& cf, const LjPair<double>& cd,
                 bool branchless, int homes, hipStream_t s) {
  if (FP64 || homes == 4)
    launch_tile_k<FP64, ENERGY, 4, LIST>(v, ff, cf, cd, branchless, s);
  else if (homes == 16)
    launch_tile_k<FP64, ENERGY, 16, LIST>(v, ff, cf, cd, branchless, s);
  else
    launch_tile_k<FP64, ENERGY, 8, LIST>(v, ff, cf, cd, branchless, s);
}

}  // namespace

int64_t lj_blocks_for_box(int kernel, int64_t n_atoms, int64_t n_cells) {
  if (kernel == 2 || kernel == 3 || kernel == 5 || kernel == 6) return (n_cells + kTileWaves - 1) / kTileWaves;
  if (kernel == 4) return (n_atoms + kLjNlBlock - 1) / kLjNlBlock;
  return (n_atoms + kLjAtomBlock - 1) / kLjAtomBlock;
}

void launch_nl_build(const Views& v, const FFDev& ff, bool fp32, int kernel, hipStream_t s, const int32_t* gate) {
  dim3 g((v.n_cell_blocks + kXcds - 1) / kXcds * kXcds), b(64 * kTileWaves);
  if (kernel == 5) {
    if (fp32)
      hipLaunchKernelGGL((k_nl_build_tile<false>), g, b, 0, s, v, ff, gate);
    else
      hipLaunchKernelGGL((k_nl_build_tile<true>), g, b, 0, s, v, ff, gate);
    return;
  }
  if (fp32)
    hipLaunchKernelGGL((k_nl_build<false, kTileHomesMixed>), g, b, 0, s, v, ff, gate);
  else
    hipLaunchKernelGGL((k_nl_build<true, 4>), g, b, 0, s, v, ff, gate);
}

// Neighbour-list forces always read the current payload (the build's right after a rebuild).
void launch_lj_nl(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, int homes, hipStream_t s) {
  const LjPair<float> cf = make_pair<float>(ff);
  const LjPair<double> cd = make_pair<double>(ff);
  const void* pay = v.pay_cur;
  if (kernel == 5) {   // per-cell lists through the cell tile, reading the current payload
    Views w = v;
    w.payload = const_cast<void*>(pay);
    if (fp32) {
      if (energy) launch_tile<false, true, true>(w, ff, cf, cd, false, homes, s);
      else launch_tile<false, false, true>(w, ff, cf, cd, false, homes, s);
    } else {
      if (energy) launch_tile<true, true, true>(w, ff, cf, cd, false, homes, s);
      else launch_tile<true, false, true>(w, ff, cf, cd, false, homes, s);
    }
    return;
  }
  dim3 g(v.n_lj_blocks), b(kLjNlBlock);
#define MDK_NL(F64, E, U) hipLaunchKernelGGL((k_lj_nl<F64, E, U>), g, b, 0, s, v, ff, cf, cd, pay)
  if (fp32) {
    if (ff.uniform_lj) { if (energy) MDK_NL(false, true, true); else MDK_NL(false, false, true); }
    else { if (energy) MDK_NL(false, true, false); else MDK_NL(false, false, false); }
  } else {
    if (ff.uniform_lj) { if (energy) MDK_NL(true, true, true); else MDK_NL(true, false, true); }
    else { if (energy) MDK_NL(true, true, false); else MDK_NL(true, false, false); }
  }
#undef MDK_NL
}

void launch_lj(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, int homes, hipStream_t s) {
  const LjPair<float> cf = make_pair<float>(ff);
  const LjPair<double> cd = make_pair<double>(ff);
  if (kernel == 6) {
    dim3 g((v.n_lj_blocks + kXcds - 1) / kXcds * kXcds), b(64 * kTileWaves);
    if (fp32) {
      if (energy) hipLaunchKernelGGL((k_lj_half<false, true>), g, b, 0, s, v, ff, cf, cd);
      else hipLaunchKernelGGL((k_lj_half<false, false>), g, b, 0, s, v, ff, cf, cd);
    } else {
      if (energy) hipLaunchKernelGGL((k_lj_half<true, true>), g, b, 0, s, v, ff, cf, cd);
      else hipLaunchKernelGGL((k_lj_half<true, false>), g, b, 0, s, v, ff, cf, cd);
    }
    const int fg = (int)std::min<int64_t>((3 * v.N + 255) / 256, 4096);
    if (fp32) hipLaunchKernelGGL(k_half_finish<float>, dim3(fg), dim3(256), 0, s, v);
    else hipLaunchKernelGGL(k_half_finish<double>, dim3(fg), dim3(256), 0, s, v);
    return;
  }
  if (kernel == 2 || kernel == 3) {
    const bool bl = kernel == 3 && fp32;
    if (fp32) {
      if (energy) launch_tile<false, true>(v, ff, cf, cd, bl, homes, s);
      else launch_tile<false, false>(v, ff, cf, cd, bl, homes, s);
    } else {
      if (energy) launch_tile<true, true>(v, ff, cf, cd, bl, homes, s);
      else launch_tile<true, false>(v, ff, cf, cd, bl, homes, s);
    }
    return;
  }
  dim3 g(v.n_lj_blocks), b(kLjAtomBlock);
  if (fp32) {
    if (energy) hipLaunchKernelGGL((k_lj_atom<false, true>), g, b, 0, s, v, ff, cf, cd);
    else hipLaunchKernelGGL((k_lj_atom<false, false>), g, b, 0, s, v, ff, cf, cd);
  } else {
    if (energy) hipLaunchKernelGGL((k_lj_atom<true, true>), g, b, 0, s, v, ff, cf, cd);
    else hipLaunchKernelGGL((k_lj_atom<true, false>), g, b, 0, s, v, ff, cf, cd);
  }
}

}  // namespace mdk
