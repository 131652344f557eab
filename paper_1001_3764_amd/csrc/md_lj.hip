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
// cell; a neighbour cell offset (ox, oy, oz) becomes the constant shift
// -(ox, oy, oz) * edge, so differences stay small and FP32 keeps ~1e-7 A.
#include "md_internal.h"

namespace mdk {
namespace {

struct alignas(32) Pay64 {
  double x, y, z, tagbits;
};

__device__ inline int32_t pay_tag(const float4& q) { return __float_as_int(q.w); }
__device__ inline int32_t pay_tag(const Pay64& q) { return (int32_t)__double_as_longlong(q.tagbits); }

__device__ inline float rcp_p(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_p(double x) { return 1.0 / x; }

__device__ inline int lane() { return (int)(threadIdx.x & 63); }

template <typename P>
struct LjPair {
  P f12[4], f6[4], e12[4], e6[4], ecut[4];
};

template <typename P>
__device__ inline P pick(const P* a, int t) {
  return t == 0 ? a[0] : (t == 1 ? a[1] : (t == 2 ? a[2] : a[3]));
}

// Lane per home atom: slot s of the sorted arrays is one lane; the lane walks the
// (2R+1)^3 cells around its own cell.
template <typename P, typename PayT, bool ENERGY>
__global__ __launch_bounds__(kLjAtomBlock) void k_lj_atom(Views v, FFDev ff, LjPair<P> cp) {
  __shared__ dd red[kLjAtomBlock / 64][3];
  const int b = v.lj_blk_box[blockIdx.x];
  const BoxDev& B = v.boxes[b];
  const int local = ((int)blockIdx.x - B.lj_blk_off) * kLjAtomBlock + (int)threadIdx.x;
  const bool active = local < B.n_atoms;
  const PayT* __restrict__ pay = static_cast<const PayT*>(v.payload);
  const int32_t* __restrict__ cstart = v.cell_start;
  const int R = v.R;
  const P rc2 = (P)ff.rc2;
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
      const P xz = (P)pi.z + (P)(-oz * B.edge[2]);
      for (int oy = -R; oy <= R; ++oy) {
        int ny = ky + oy;
        ny += ny < 0 ? M1 : 0;
        ny -= ny >= M1 ? M1 : 0;
        const P xy = (P)pi.y + (P)(-oy * B.edge[1]);
        for (int ox = -R; ox <= R; ++ox) {
          int nx = kx + ox;
          nx += nx < 0 ? M0 : 0;
          nx -= nx >= M0 ? M0 : 0;
          const P xx = (P)pi.x + (P)(-ox * B.edge[0]);
          const int nc = B.cell_off + nx + M0 * (ny + M1 * nz);
          const int t1 = cstart[nc + 1];
          for (int t = cstart[nc]; t < t1; ++t) {
            const PayT pj = pay[t];
            const int32_t tj = pay_tag(pj);
            const P dx = xx - (P)pj.x, dy = xy - (P)pj.y, dz = xz - (P)pj.z;
            const P r2 = dx * dx + dy * dy + dz * dz;
            const bool excl = (uint32_t)(tag_index(tj) - lo) <= span;
            if (r2 < rc2 && !excl) {
              const int tt = ff.uniform_lj ? 0 : ti * 2 + tag_type(tj);
              const P r2i = rcp_p(r2);
              const P r6 = r2i * r2i * r2i;
              const P ffs = r2i * r6 * (pick(cp.f12, tt) * r6 - pick(cp.f6, tt));
              fx += ffs * dx;
              fy += ffs * dy;
              fz += ffs * dz;
              if (ENERGY) {
                const P en = r6 * (pick(cp.e12, tt) * r6 - pick(cp.e6, tt));
                e += (double)en;
                es += (double)en - (double)pick(cp.ecut, tt);
                w += (double)(ffs * r2);
              }
            }
          }
        }
      }
    }
    P* f = static_cast<P*>(v.f_lj);
    f[i] = fx;
    f[v.N + i] = fy;
    f[2 * v.N + i] = fz;
  }
  if (ENERGY) {
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
        for (int wv = 1; wv < kLjAtomBlock / 64; ++wv) s = dd_add(s, red[wv][k]);
        v.part_lj[(int64_t)blockIdx.x * 3 + k] = s;
      }
  }
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

}  // namespace

int64_t lj_blocks_for_box(int kernel, int64_t n_atoms, int64_t n_cells) {
  (void)kernel;
  (void)n_cells;
  return (n_atoms + kLjAtomBlock - 1) / kLjAtomBlock;
}

void launch_lj(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, hipStream_t s) {
  (void)kernel;
  dim3 g(v.n_lj_blocks), b(kLjAtomBlock);
  if (fp32) {
    const LjPair<float> cp = make_pair<float>(ff);
    if (energy)
      hipLaunchKernelGGL((k_lj_atom<float, float4, true>), g, b, 0, s, v, ff, cp);
    else
      hipLaunchKernelGGL((k_lj_atom<float, float4, false>), g, b, 0, s, v, ff, cp);
  } else {
    const LjPair<double> cp = make_pair<double>(ff);
    if (energy)
      hipLaunchKernelGGL((k_lj_atom<double, Pay64, true>), g, b, 0, s, v, ff, cp);
    else
      hipLaunchKernelGGL((k_lj_atom<double, Pay64, false>), g, b, 0, s, v, ff, cp);
  }
}

}  // namespace mdk
