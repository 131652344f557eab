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
// Two kernels:
//   k_lj_atom  one lane per home atom walking the stencil cells (the paper's shape);
//   k_lj_tile  one wavefront per home cell: the cell's atoms are wave-uniform (KMAX
//              at a time) and candidate atoms stream across the lanes, two stencil
//              rows at a time (one per 32-lane half), so lanes stay busy whatever
//              the cell occupancy.
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

// Values that are the same on every lane, moved to scalar registers.
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline double uni(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename P>
struct LjPair {
  P f12[4], f6[4], e12[4], e6[4], ecut[4];
};

template <typename P>
__device__ inline P pick(const P* a, int t) {
  return t == 0 ? a[0] : (t == 1 ? a[1] : (t == 2 ? a[2] : a[3]));
}

// One pair, mixed precision.  d* are exact fixed-point differences x_i - x_j; the force
// accumulated in a* is in units of 2^25 (the caller scales the final sum by 2^-25).
// BRANCHLESS evaluates the force for every lane and zeroes it outside the cutoff.
template <bool ENERGY, bool BRANCHLESS = false>
__device__ __forceinline__ void pair_fix(int dqx, int dqy, int dqz, bool keep, float rc2s, float f12,
                                         float f6, float e12, float e6, float ecut, float& ax, float& ay,
                                         float& az, double& e, double& es, double& w) {
  const float dx = (float)dqx, dy = (float)dqy, dz = (float)dqz;
  const float r2s = dx * dx + dy * dy + dz * dz;     // units of 2^-50 A^2
  const bool hit = keep && r2s < rc2s;
  if (BRANCHLESS || hit) {
    const float r2 = r2s * kInvFix2F;
    const float r2i = rcp_f(r2);
    const float r6 = r2i * r2i * r2i;
    const float g = r6 * (f12 * r6 - f6);             // = F . r, kcal/mol
    float ffs = g * r2i;
    if (BRANCHLESS) ffs = hit ? ffs : 0.0f;
    ax += ffs * dx;
    ay += ffs * dy;
    az += ffs * dz;
    if (ENERGY && hit) {
      const float en = r6 * (e12 * r6 - e6);
      e += (double)en;
      es += (double)en - (double)ecut;
      w += (double)g;
    }
  }
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
    for (int off = 32; off > 0; off >>= 1) {
      dd o{__shfl_xor(q[k].hi, off), __shfl_xor(q[k].lo, off)};
      q[k] = dd_add(q[k], o);
    }
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
  const float rc2s = (float)(ff.rc2 * kFix * kFix);
  double e = 0.0, es = 0.0, w = 0.0;
  if (active) {
    const int64_t s = (int64_t)B.atom_off + local;
    const PayT pi = pay[s];
    const int32_t tag = pay_tag(pi);
    const int32_t i = tag_index(tag);
    const int ti = tag_type(tag);
    const int32_t cs = i - i % ff.chain_len;
    const int32_t lo = max(i - ff.excl, cs);
    const int32_t hi = min(i + ff.excl, cs + ff.chain_len - 1);
    const uint32_t span = (uint32_t)(hi - lo);
    const int c = v.scell[s] - B.cell_off;
    const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
    const int kx = c % M0, ky = (c / M0) % M1, kz = c / (M0 * M1);
    P fx = 0, fy = 0, fz = 0;
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
              pair_fix<ENERGY>(hx - pj.x, hy - pj.y, hz - pj.z, keep, rc2s, pick(cf.f12, tt), pick(cf.f6, tt),
                               pick(cf.e12, tt), pick(cf.e6, tt), pick(cf.ecut, tt), fx, fy, fz, e, es, w);
            }
          }
        }
      }
    }
    if constexpr (!FP64) {
      fx *= kInvFixF;
      fy *= kInvFixF;
      fz *= kInvFixF;
    }
    P* f = static_cast<P*>(v.f_lj);
    f[i] = fx;
    f[v.N + i] = fy;
    f[2 * v.N + i] = fz;
  }
  if (ENERGY) block_energy<kLjAtomBlock / 64>(e, es, w, red, v.part_lj + (int64_t)blockIdx.x * 3);
}

// ---------------------------------------------------------------------------------
// Cell tile: wave = one home cell.
struct Piece {
  int start, count;   // sorted-array range of consecutive cells of one stencil row
  int ox0, cx0;       // x-offset of the first cell from the home cell, and its x index
  int oy, oz;         // row offsets
};
constexpr int kMaxPieces = 2 * (2 * kTileMaxR + 1) * (2 * kTileMaxR + 1);

template <bool FP64, bool ENERGY, bool UNI, int KMAX, bool BRANCHLESS>
__global__ __launch_bounds__(64 * kTileWaves) void k_lj_tile(Views v, FFDev ff, LjPair<float> cf,
                                                             LjPair<double> cd) {
  using PayT = std::conditional_t<FP64, Pay64, int4>;
  using P = std::conditional_t<FP64, double, float>;
  using Q = std::conditional_t<FP64, double, int>;     // coordinate type
  __shared__ Piece pieces[kTileWaves][kMaxPieces];
  __shared__ int npieces[kTileWaves];
  __shared__ dd red[kTileWaves][3];

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int ln = lane(), half = ln >> 5, hl = ln & 31;
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
  // home cells (a slab of the box) so its L2 holds one neighbourhood of the payload.
  const int per_xcd = (int)gridDim.x / kXcds;
  const int blk = ((int)blockIdx.x % kXcds) * per_xcd + (int)blockIdx.x / kXcds;
  if (blk >= v.n_lj_blocks) return;
  const int b = v.lj_blk_box[blk];
  const BoxDev& B = v.boxes[b];
  const int lc = (blk - B.lj_blk_off) * kTileWaves + wave;   // home cell within the box
  const bool wact = lc < B.n_cells;
  const int R = v.R, W = 2 * R + 1;
  const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
  const int kx = lc % M0, ky = (lc / M0) % M1, kz = lc / (M0 * M1);
  const int32_t* __restrict__ cs = v.cell_start;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);

  // ---- stencil rows -> contiguous pieces of the sorted arrays (split at the x wrap)
  {
    Piece p1{0, 0, 0, 0, 0, 0}, p2{0, 0, 0, 0, 0, 0};
    int has = 0;
    if (wact && ln < W * W) {
      const int oy = ln % W - R, oz = ln / W - R;
      int ny = ky + oy;
      ny += ny < 0 ? M1 : 0;
      ny -= ny >= M1 ? M1 : 0;
      int nz = kz + oz;
      nz += nz < 0 ? M2 : 0;
      nz -= nz >= M2 ? M2 : 0;
      const int row = B.cell_off + M0 * (ny + M1 * nz);
      const int xa = kx - R, xb = kx + R;
      if (xa >= 0 && xb < M0) {
        p1 = Piece{cs[row + xa], cs[row + xb + 1] - cs[row + xa], -R, xa, oy, oz};
        has = 1;
      } else if (xa < 0) {
        p1 = Piece{cs[row + xa + M0], cs[row + M0] - cs[row + xa + M0], -R, xa + M0, oy, oz};
        p2 = Piece{cs[row], cs[row + xb + 1] - cs[row], -kx, 0, oy, oz};
        has = 2;
      } else {
        p1 = Piece{cs[row + xa], cs[row + M0] - cs[row + xa], -R, xa, oy, oz};
        p2 = Piece{cs[row], cs[row + xb - M0 + 1] - cs[row], M0 - kx, 0, oy, oz};
        has = 2;
      }
    }
    const uint64_t m1 = __ballot(has >= 1), m2 = __ballot(has == 2);
    const uint64_t below = (1ull << ln) - 1ull;
    const int idx = __popcll(m1 & below) + __popcll(m2 & below);
    if (has >= 1) pieces[wave][idx] = p1;
    if (has == 2) pieces[wave][idx + 1] = p2;
    if (ln == 0) npieces[wave] = __popcll(m1) + __popcll(m2);
  }
  __syncthreads();

  double e = 0.0, es = 0.0, w = 0.0;
  if (wact) {
    const int hs = __builtin_amdgcn_readfirstlane(cs[B.cell_off + lc]);
    const int hn = __builtin_amdgcn_readfirstlane(cs[B.cell_off + lc + 1]) - hs;
    const int np = __builtin_amdgcn_readfirstlane(npieces[wave]);
    const float rc2s = (float)(ff.rc2 * kFix * kFix);
    const Q ex = FP64 ? (Q)0 : (Q)B.edge_q[0];
    for (int g0 = 0; g0 < hn; g0 += KMAX) {
      const int kc = min(KMAX, hn - g0);
      Q hx[KMAX], hy[KMAX], hz[KMAX];
      int32_t lo[KMAX], hti[KMAX];
      uint32_t span[KMAX];
      P ax[KMAX], ay[KMAX], az[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        ax[k] = ay[k] = az[k] = (P)0;
        if (k < kc) {
          const PayT q = pay[hs + g0 + k];
          // FP64 homes go to scalar registers (measured faster); mixed ones stay in
          // vector registers, where the scalar budget would otherwise spill
          if constexpr (FP64) {
            hx[k] = uni(q.x);
            hy[k] = uni(q.y);
            hz[k] = uni(q.z);
          } else {
            hx[k] = q.x;
            hy[k] = q.y;
            hz[k] = q.z;
          }
          const int32_t tag = FP64 ? uni(pay_tag(q)) : pay_tag(q);
          const int32_t i = tag_index(tag);
          const int32_t c0 = i - i % ff.chain_len;
          lo[k] = max(i - ff.excl, c0);
          span[k] = (uint32_t)(min(i + ff.excl, c0 + ff.chain_len - 1) - lo[k]);
          hti[k] = tag_type(tag);
        } else {
          hx[k] = hy[k] = hz[k] = (Q)0;
          lo[k] = 0;
          span[k] = 0;
          hti[k] = 0;
        }
      }
      // two candidate streams, one per 32-lane half: pieces half, half+2, half+4, ...
      int p = half, o = 0;
      while (true) {
        const bool hv = p < np;
        if (__ballot(hv) == 0) break;
        Piece pc{0, 0, 0, 0, 0, 0};
        if (hv) pc = pieces[wave][p];
        const bool act = hv && (o + hl < pc.count);
        Q jx = (Q)0, jy = (Q)0, jz = (Q)0;
        int32_t jt = 0;
        if (act) {
          const PayT q = pay[pc.start + o + hl];
          jt = pay_tag(q);
          const int ox = pc.ox0 + ((tag_cx(jt) - pc.cx0) & 7);
          // candidate in the home cell's frame
          if constexpr (FP64) {
            jx = q.x + ox * B.edge[0];
            jy = q.y + pc.oy * B.edge[1];
            jz = q.z + pc.oz * B.edge[2];
          } else {
            jx = q.x + ox * ex;
            jy = q.y + pc.oy * B.edge_q[1];
            jz = q.z + pc.oz * B.edge_q[2];
          }
        }
        const int32_t jidx = tag_index(jt);
        const int jtype = tag_type(jt);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          if (k < kc) {
            const bool keep = act && (uint32_t)(jidx - lo[k]) > span[k];
            const int tt = UNI ? 0 : hti[k] * 2 + jtype;
            if constexpr (FP64)
              pair_f64<ENERGY>(hx[k] - jx, hy[k] - jy, hz[k] - jz, keep, ff.rc2, pick(cd.f12, tt),
                               pick(cd.f6, tt), pick(cd.e12, tt), pick(cd.e6, tt), pick(cd.ecut, tt), ax[k],
                               ay[k], az[k], e, es, w);
            else
              pair_fix<ENERGY, BRANCHLESS>(hx[k] - jx, hy[k] - jy, hz[k] - jz, keep, rc2s, pick(cf.f12, tt),
                                           pick(cf.f6, tt), pick(cf.e12, tt), pick(cf.e6, tt),
                                           pick(cf.ecut, tt), ax[k], ay[k], az[k], e, es, w);
          }
        }
        o += 32;
        if (hv && o >= pc.count) {
          p += 2;
          o = 0;
        }
      }
      // sum each home atom's partial forces over the 64 lanes (fixed butterfly order)
      P* f = static_cast<P*>(v.f_lj);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < kc) {
          P sx = ax[k], sy = ay[k], sz = az[k];
          for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off);
            sy += __shfl_xor(sy, off);
            sz += __shfl_xor(sz, off);
          }
          if constexpr (!FP64) {
            sx *= kInvFixF;
            sy *= kInvFixF;
            sz *= kInvFixF;
          }
          if (ln == k) {
            const int32_t i = tag_index(pay_tag(pay[hs + g0 + k]));
            f[i] = sx;
            f[v.N + i] = sy;
            f[2 * v.N + i] = sz;
          }
        }
      }
    }
  }
  if (ENERGY) block_energy<kTileWaves>(e, es, w, red, v.part_lj + (int64_t)blk * 3);
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
  return c;
}

template <bool FP64, bool ENERGY>
void launch_tile(const Views& v, const FFDev& ff, const LjPair<float>& cf, const LjPair<double>& cd,
                 bool branchless, hipStream_t s) {
  dim3 g((v.n_lj_blocks + kXcds - 1) / kXcds * kXcds), b(64 * kTileWaves);
  constexpr int K = FP64 ? 4 : 8;
  if (ff.uniform_lj) {
    if (branchless)
      hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, true, K, true>), g, b, 0, s, v, ff, cf, cd);
    else
      hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, true, K, false>), g, b, 0, s, v, ff, cf, cd);
  } else {
    hipLaunchKernelGGL((k_lj_tile<FP64, ENERGY, false, K, false>), g, b, 0, s, v, ff, cf, cd);
  }
}

}  // namespace

int64_t lj_blocks_for_box(int kernel, int64_t n_atoms, int64_t n_cells) {
  if (kernel == 2 || kernel == 3) return (n_cells + kTileWaves - 1) / kTileWaves;
  return (n_atoms + kLjAtomBlock - 1) / kLjAtomBlock;
}

void launch_lj(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, hipStream_t s) {
  const LjPair<float> cf = make_pair<float>(ff);
  const LjPair<double> cd = make_pair<double>(ff);
  if (kernel == 2 || kernel == 3) {
    const bool bl = kernel == 3 && fp32;
    if (fp32) {
      if (energy) launch_tile<false, true>(v, ff, cf, cd, bl, s);
      else launch_tile<false, false>(v, ff, cf, cd, bl, s);
    } else {
      if (energy) launch_tile<true, true>(v, ff, cf, cd, bl, s);
      else launch_tile<true, false>(v, ff, cf, cd, bl, s);
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
