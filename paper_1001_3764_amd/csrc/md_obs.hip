// Structural observables of Section 5 for gfx950: the pair-distance histogram behind the
// radial distribution function (Fig. 10), the dihedral-angle distribution and trans /
// gauche fractions (Figs. 9, 15), and per-chain radius of gyration and end-to-end vector
// (Figs. 8, 12).
//
//   k_obs_pairs      one lane per atom of the sorted order: its own cell (the atoms after it
//                    in the sorted order) and the forward half of the current grid's stencil
//                    (with at least 2R + 1 cells per dimension no pair of cells is reached from
//                    both sides), so every unordered non-excluded pair is counted once; the
//                    bin is decided in FP64 on r^2 against squared edges, so the counts are
//                    exact integers; a block histogram in LDS (integer atomics: the counts
//                    do not depend on their order), one row of block partials per block
//   k_obs_dihedrals  one lane per dihedral: the IUPAC angle, its bin and its class
//   k_obs_reduce     per bin, the block partials in block order (64-bit)
//   k_obs_chains     one wavefront per chain: the chain unwrapped bond by bond (a wave
//                    prefix sum per 64 atoms), centre of mass, then R_g^2 and R_ee
//   k_ree,           the end-to-end vector autocorrelation (Fig. 8): each chain's R_ee
//   k_ree_reduce     against the one stored at the reference time, summed per box
#include "md_internal.h"

namespace mdk {
namespace {

__device__ inline int lane() { return (int)(threadIdx.x & 63); }

// minimum image of one coordinate difference, no fused multiply-add
__device__ inline double mi_rn(double t, double L, double invL) {
  return __dadd_rn(t, -__dmul_rn(L, rint(__dmul_rn(t, invL))));
}

// the largest k with (k dr)^2 <= r2 (r2 below the last edge)
__device__ inline int distance_bin(double r2, double dr, int n_bins) {
  int k = (int)(sqrt(r2) / dr);
  if (k > n_bins - 1) k = n_bins - 1;
  while (k > 0 && r2 < __dmul_rn(__dmul_rn((double)k, dr), __dmul_rn((double)k, dr))) --k;
  while (k + 1 < n_bins && r2 >= __dmul_rn(__dmul_rn((double)(k + 1), dr), __dmul_rn((double)(k + 1), dr))) ++k;
  return k;
}

__global__ __launch_bounds__(kAtomBlock) void k_obs_pairs(Views v, int b, int chain_len, int excl, double dr,
                                                        int n_bins, uint32_t* part) {
  __shared__ uint32_t hist[kMaxObsBins];
  for (int k = (int)threadIdx.x; k < n_bins; k += kAtomBlock) hist[k] = 0;
  __syncthreads();
  const BoxDev& B = v.boxes[b];
  const double rmax2 = __dmul_rn(__dmul_rn((double)n_bins, dr), __dmul_rn((double)n_bins, dr));
  const int64_t N = v.N;
  const int R = v.R, W = 2 * R + 1;
  const int M0 = B.M[0], M1 = B.M[1], M2 = B.M[2];
  for (int64_t s = B.atom_off + (int64_t)blockIdx.x * kAtomBlock + threadIdx.x; s < B.atom_off + B.n_atoms;
       s += (int64_t)gridDim.x * kAtomBlock) {
    const int32_t i = v.cell_atoms[s];
    const int lc = v.scell[s] - B.cell_off;
    const Cell3 k3 = cell_coords(lc, B);
    const double xi = v.pos[i], yi = v.pos[N + i], zi = v.pos[2 * N + i];
    const int32_t ci = i / chain_len;
    const int ctr = (W * W * W - 1) / 2;   // the cell itself; codes above it are the forward half
    for (int code = ctr; code < W * W * W; ++code) {
      const Cell3 o = stencil_offset(code, R);
      int nx = k3.x + o.x, ny = k3.y + o.y, nz = k3.z + o.z;
      nx += nx < 0 ? M0 : 0;
      nx -= nx >= M0 ? M0 : 0;
      ny += ny < 0 ? M1 : 0;
      ny -= ny >= M1 ? M1 : 0;
      nz += nz < 0 ? M2 : 0;
      nz -= nz >= M2 ? M2 : 0;
      const int c = B.cell_off + nx + M0 * (ny + M1 * nz);
      const int32_t e = v.cell_start[c + 1];
      for (int32_t t = code == ctr ? (int32_t)s + 1 : v.cell_start[c]; t < e; ++t) {
        const int32_t j = v.cell_atoms[t];
        if (j / chain_len == ci && abs(j - i) <= excl) continue;
        const double dx = mi_rn(__dadd_rn(xi, -v.pos[j]), B.L[0], B.invL[0]);
        const double dy = mi_rn(__dadd_rn(yi, -v.pos[N + j]), B.L[1], B.invL[1]);
        const double dz = mi_rn(__dadd_rn(zi, -v.pos[2 * N + j]), B.L[2], B.invL[2]);
        const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        if (r2 < rmax2) atomicAdd(&hist[distance_bin(r2, dr, n_bins)], 1u);
      }
    }
  }
  __syncthreads();
  for (int k = (int)threadIdx.x; k < n_bins; k += kAtomBlock) part[(int64_t)blockIdx.x * kMaxObsBins + k] = hist[k];
}

// IUPAC dihedral angle of sites (p, p+1, p+2, p+3), bonds minimum-imaged
__device__ inline double dihedral_phi(const Views& v, const BoxDev& B, int64_t p) {
  const int64_t N = v.N;
  double s[4][3];
  for (int q = 0; q < 3; ++q) s[0][q] = v.pos[q * N + p];
  for (int a = 1; a < 4; ++a)
    for (int q = 0; q < 3; ++q)
      s[a][q] = s[a - 1][q] + mi_rn(v.pos[q * N + p + a] - v.pos[q * N + p + a - 1], B.L[q], B.invL[q]);
  double F[3], G[3], H[3];
  for (int q = 0; q < 3; ++q) {
    F[q] = s[0][q] - s[1][q];
    G[q] = s[1][q] - s[2][q];
    H[q] = s[3][q] - s[2][q];
  }
  const double A[3] = {F[1] * G[2] - F[2] * G[1], F[2] * G[0] - F[0] * G[2], F[0] * G[1] - F[1] * G[0]};
  const double Bv[3] = {H[1] * G[2] - H[2] * G[1], H[2] * G[0] - H[0] * G[2], H[0] * G[1] - H[1] * G[0]};
  const double BA[3] = {Bv[1] * A[2] - Bv[2] * A[1], Bv[2] * A[0] - Bv[0] * A[2], Bv[0] * A[1] - Bv[1] * A[0]};
  const double lA = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
  const double lB = sqrt(Bv[0] * Bv[0] + Bv[1] * Bv[1] + Bv[2] * Bv[2]);
  const double lG = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
  const double c = (A[0] * Bv[0] + A[1] * Bv[1] + A[2] * Bv[2]) / (lA * lB);
  const double sn = (BA[0] * G[0] + BA[1] * G[1] + BA[2] * G[2]) / (lA * lB * lG);
  return atan2(sn, c);
}

// bins [0, n_bins): the angle histogram; n_bins, n_bins + 1, n_bins + 2: trans, gauche+, gauche-
__global__ __launch_bounds__(kAtomBlock) void k_obs_dihedrals(Views v, int b, int chain_len, int n_bins,
                                                            uint32_t* part) {
  __shared__ uint32_t hist[kMaxObsBins];
  const int nb = n_bins + 3;
  for (int k = (int)threadIdx.x; k < nb; k += kAtomBlock) hist[k] = 0;
  __syncthreads();
  const BoxDev& B = v.boxes[b];
  const double pi = 3.141592653589793, two_pi = 2.0 * pi, third = two_pi / 3.0, scale = n_bins / two_pi;
  for (int64_t t = (int64_t)blockIdx.x * kAtomBlock + threadIdx.x; t < B.n_atoms; t += (int64_t)gridDim.x * kAtomBlock) {
    if (t % chain_len + 3 >= chain_len) continue;
    const double phi = dihedral_phi(v, B, B.atom_off + t);
    if (n_bins > 0) {
      int k = (int)floor((phi + pi) * scale);
      k = k > n_bins - 1 ? n_bins - 1 : (k < 0 ? 0 : k);
      atomicAdd(&hist[k], 1u);
    }
    atomicAdd(&hist[n_bins + (fabs(phi) > third ? 0 : (phi >= 0.0 ? 1 : 2))], 1u);
  }
  __syncthreads();
  for (int k = (int)threadIdx.x; k < nb; k += kAtomBlock) part[(int64_t)blockIdx.x * kMaxObsBins + k] = hist[k];
}

__global__ __launch_bounds__(256) void k_obs_reduce(const uint32_t* part, int n_blocks, int n_bins,
                                                   unsigned long long* out) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k >= n_bins) return;
  unsigned long long s = 0;
  for (int q = 0; q < n_blocks; ++q) s += part[(int64_t)q * kMaxObsBins + k];
  out[k] = s;
}

__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ inline double wave_inclusive_scan(double x) {
  const int ln = lane();
  for (int d = 1; d < 64; d <<= 1) {
    const double y = __shfl_up(x, d);
    if (ln >= d) x += y;
  }
  return x;
}

// One wavefront per chain of box b.  Pass 1: unwrapped positions u_p = x_0 + sum of the
// minimum-imaged bonds up to p, mass-weighted sums; pass 2: sum m |u - u_cm|^2.
__global__ __launch_bounds__(256) void k_obs_chains(Views v, FFDev ff, int b, int chain_len, double* out) {
  const BoxDev& B = v.boxes[b];
  const int n_chains = B.n_atoms / chain_len;
  const int ch = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (ch >= n_chains) return;
  const int ln = lane();
  const int64_t N = v.N;
  const int64_t a0 = (int64_t)B.atom_off + (int64_t)ch * chain_len;
  double x0[3];
  for (int q = 0; q < 3; ++q) x0[q] = v.pos[q * N + a0];
  double cm[3] = {0.0, 0.0, 0.0}, msum = 0.0, rg = 0.0, ree[3] = {0.0, 0.0, 0.0};
  for (int pass = 0; pass < 2; ++pass) {
    double carry[3] = {0.0, 0.0, 0.0};
    double acc[3] = {0.0, 0.0, 0.0}, macc = 0.0, racc = 0.0;
    for (int p0 = 0; p0 < chain_len; p0 += 64) {
      const int p = p0 + ln;
      const bool in = p < chain_len;
      double u[3];
      for (int q = 0; q < 3; ++q) {
        double d = 0.0;
        if (in && p > 0) d = mi_rn(v.pos[q * N + a0 + p] - v.pos[q * N + a0 + p - 1], B.L[q], B.invL[q]);
        const double sc = wave_inclusive_scan(d);
        u[q] = x0[q] + (carry[q] + sc);
        carry[q] += __shfl(sc, 63);
      }
      if (in) {
        const double m = ff.mass[v.type[a0 + p]];
        if (pass == 0) {
          macc += m;
          for (int q = 0; q < 3; ++q) acc[q] += m * u[q];
        } else {
          double d2 = 0.0;
          for (int q = 0; q < 3; ++q) d2 += (u[q] - cm[q]) * (u[q] - cm[q]);
          racc += m * d2;
        }
      }
    }
    if (pass == 0) {
      msum = wave_sum(macc);
      for (int q = 0; q < 3; ++q) {
        cm[q] = wave_sum(acc[q]) / msum;
        ree[q] = carry[q];
      }
    } else {
      rg = wave_sum(racc) / msum;
    }
  }
  if (ln == 0) {
    const int64_t c = (int64_t)B.atom_off / chain_len + ch;
    out[4 * c] = rg;
    for (int q = 0; q < 3; ++q) out[4 * c + 1 + q] = ree[q];
  }
}

// End-to-end vector autocorrelation (Fig. 8).  One wavefront per chain of box b: R, the sum
// of the chain's minimum-imaged bonds (each lane sums every 64th bond, then a fixed-order wave
// sum).  REF: store R as the reference ree0[c]; otherwise write the chain's terms
// part[2 c] = R . ree0[c] and part[2 c + 1] = |ree0[c]|^2.
template <bool REF>
__global__ __launch_bounds__(256) void k_ree(Views v, int b, int chain_len, double* ree0, double* part) {
  const BoxDev& B = v.boxes[b];
  const int n_chains = B.n_atoms / chain_len;
  const int ch = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (ch >= n_chains) return;
  const int ln = lane();
  const int64_t N = v.N;
  const int64_t a0 = (int64_t)B.atom_off + (int64_t)ch * chain_len;
  double r[3] = {0.0, 0.0, 0.0};
  for (int p = 1 + ln; p < chain_len; p += 64)
    for (int q = 0; q < 3; ++q)
      r[q] += mi_rn(__dadd_rn(v.pos[q * N + a0 + p], -v.pos[q * N + a0 + p - 1]), B.L[q], B.invL[q]);
  for (int q = 0; q < 3; ++q) r[q] = wave_sum(r[q]);
  if (ln != 0) return;
  const int64_t c = (int64_t)B.atom_off / chain_len + ch;
  if (REF) {
    for (int q = 0; q < 3; ++q) ree0[3 * c + q] = r[q];
  } else {
    const double* r0 = ree0 + 3 * c;
    part[2 * c] = r[0] * r0[0] + r[1] * r0[1] + r[2] * r0[2];
    part[2 * c + 1] = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
  }
}

// Box b's autocorrelation: the chain terms of k_ree summed in chain order as double-double
// (each thread a contiguous run of chains, then the runs in thread order), out[b] = num / den.
__global__ __launch_bounds__(256) void k_ree_reduce(Views v, int b, int chain_len, const double* part,
                                                    double* out) {
  __shared__ dd sh[256][2];
  const BoxDev& B = v.boxes[b];
  const int64_t c0 = (int64_t)B.atom_off / chain_len;
  const int64_t n = B.n_atoms / chain_len;
  const int64_t per = (n + 255) / 256;
  dd num = dd_from(0.0), den = dd_from(0.0);
  for (int64_t c = (int64_t)threadIdx.x * per; c < min(n, ((int64_t)threadIdx.x + 1) * per); ++c) {
    num = dd_add(num, dd_from(part[2 * (c0 + c)]));
    den = dd_add(den, dd_from(part[2 * (c0 + c) + 1]));
  }
  sh[threadIdx.x][0] = num;
  sh[threadIdx.x][1] = den;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < 256; ++t) {
      num = dd_add(num, sh[t][0]);
      den = dd_add(den, sh[t][1]);
    }
    out[b] = (num.hi + num.lo) / (den.hi + den.lo);
  }
}

int obs_blocks(int64_t n) {
  const int64_t g = (n + kAtomBlock - 1) / kAtomBlock;
  return (int)(g < 1 ? 1 : (g > kObsBlocks ? kObsBlocks : g));
}

}  // namespace

void launch_obs_pairs(const Views& v, int b, int64_t n_atoms, int chain_len, int excl, double dr, int n_bins,
                      unsigned long long* out, hipStream_t s) {
  const int g = obs_blocks(n_atoms);
  hipLaunchKernelGGL(k_obs_pairs, dim3(g), dim3(kAtomBlock), 0, s, v, b, chain_len, excl, dr, n_bins, v.obs_part);
  hipLaunchKernelGGL(k_obs_reduce, dim3((n_bins + 255) / 256), dim3(256), 0, s, (const uint32_t*)v.obs_part, g,
                     n_bins, out);
}

void launch_obs_dihedrals(const Views& v, int b, int64_t n_atoms, int chain_len, int n_bins,
                          unsigned long long* out, hipStream_t s) {
  const int g = obs_blocks(n_atoms);
  hipLaunchKernelGGL(k_obs_dihedrals, dim3(g), dim3(kAtomBlock), 0, s, v, b, chain_len, n_bins, v.obs_part);
  hipLaunchKernelGGL(k_obs_reduce, dim3((n_bins + 3 + 255) / 256), dim3(256), 0, s, (const uint32_t*)v.obs_part,
                     g, n_bins + 3, out);
}

void launch_obs_chains(const Views& v, const FFDev& ff, int b, int64_t n_chains, int chain_len, double* out,
                       hipStream_t s) {
  const int64_t threads = n_chains * 64;
  hipLaunchKernelGGL(k_obs_chains, dim3((int)((threads + 255) / 256)), dim3(256), 0, s, v, ff, b, chain_len, out);
}

void launch_ree(const Views& v, int b, int64_t n_chains, int chain_len, bool reference, double* out, hipStream_t s) {
  const dim3 g((unsigned)((n_chains * 64 + 255) / 256)), blk(256);
  if (reference) {
    hipLaunchKernelGGL(k_ree<true>, g, blk, 0, s, v, b, chain_len, v.ree0, v.ree_part);
  } else {
    hipLaunchKernelGGL(k_ree<false>, g, blk, 0, s, v, b, chain_len, v.ree0, v.ree_part);
    hipLaunchKernelGGL(k_ree_reduce, dim3(1), dim3(256), 0, s, v, b, chain_len, (const double*)v.ree_part, out);
  }
}

}  // namespace mdk
