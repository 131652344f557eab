// Bin rebuild, bonded forces, integration and reductions for gfx950 (wave64).
//
// Bin rebuild (Section 3.1; the paper's atomic insertion gives each atom a slot in
// its cell but an unspecified order -- here that slot is followed by a rank pass so
// the cell lists come out in ascending atom order, the same every run):
//   k_bin_count     wrap, cell index, slot = atomic count (one atomic per distinct
//                   cell per wavefront, all issued at once, lanes ranked with
//                   ballot/popcount)
//   k_scan_tiles    the total count of each tile of cells (grids of more than
//                   kScanOnePass tiles)
//   k_scan          cell_start = exclusive prefix sum of the counts (each tile's offset is
//                   the sum of the totals of the tiles before it, or on small grids of
//                   their counts)
//   k_scatter       unordered lists: tmp[cell_start[c] + slot] = atom
//   k_rank_payload  rank inside the cell = number of smaller atom indices in it;
//                   writes the ordered list and the cell-centre-relative payload
// Bonded terms (Section 3.3, Eqs. 4-6): each term is computed once by one lane, its
// per-atom forces go to LDS, and every atom gathers the terms touching it in a fixed
// order (no doubled/tripled/quadrupled work, no atomics, bitwise reproducible).
// Update (Section 3.4): velocity Verlet half-kicks and drift in FP64 with Berendsen
// scaling, or the paper's leap-frog with the Nose-Hoover extended system; optional
// removal of each box's centre-of-mass velocity (Section 3); all sums as double-double.
// Whatever a step's sums decide (the Berendsen factor, the Nose-Hoover friction, the
// centre-of-mass velocity) is applied by the next step's first kernel, so a step needs
// no grid-wide synchronisation beyond kernel boundaries.
#include "md_internal.h"

#include <type_traits>

namespace mdk {
namespace {

struct alignas(32) Pay64 {
  double x, y, z, tagbits;
};

__device__ inline double wrap_coord(double x, double L, double invL) {
  if (x >= 0.0 && x < L) return x;
  double s = floor(x * invL);
  double y = fma(-s, L, x);
  if (y >= L) y -= L;
  if (y < 0.0) y += L;
  return y;
}

__device__ inline int cell_coord(double x, double cinv, int M) {
  double f = floor(x * cinv);
  if (f < 0.0) return 0;
  if (f > (double)(M - 1)) return M - 1;
  return (int)f;
}

__device__ inline int lane() { return (int)(threadIdx.x & 63); }

// The velocity update of both integrators, v <- post * (pre * (v - u) + h f), with the
// per-box factors the last reduction left (ThermoSlot) and h = k dt a / F.
struct Kick {
  double pre, post, ux, uy, uz;
};
__device__ inline Kick load_kick(const Views& v, int b) {
  const double* t = v.thermo + (int64_t)b * kThermo;
  return Kick{t[kThPre], t[kThPost], t[kThU], t[kThU + 1], t[kThU + 2]};
}

// Slot of this lane's atom inside its cell.  Lanes are grouped by cell in a loop with
// no memory access (one ballot per distinct cell); then the first lane of every group adds
// the group's size to the cell's count, all groups in one atomic instruction (one round
// trip per wavefront), and each lane takes base + its rank in the group (lane order).
__device__ inline int aggregated_slot(int32_t* cnt, int c, bool active) {
  uint64_t pending = __ballot(active);
  const int ln = lane();
  const uint64_t below = (1ull << ln) - 1ull;
  int leader = ln, rank = 0, size = 0;
  while (pending) {
    const int l = __ffsll((unsigned long long)pending) - 1;
    const int lc = __builtin_amdgcn_readlane(c, l);
    const bool mine = active && c == lc;
    const uint64_t grp = __ballot(mine);
    if (mine) {
      leader = l;
      rank = __popcll(grp & below);
      size = __popcll(grp);
    }
    pending &= ~grp;
  }
  int base = 0;
  if (active && ln == leader) base = atomicAdd(&cnt[c], size);
  base = __shfl(base, leader);
  return base + rank;
}


// kdt: dt / 2 (velocity Verlet half kick) or dt (leap-frog)
template <typename F, bool KICK>
__global__ __launch_bounds__(kAtomBlock) void k_bin_count(Views v, const F* __restrict__ f, double dt,
                                                        double kdt, FFDev ff, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;   // neighbour-list mode: no rebuild this step
  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int local = ((int)blockIdx.x - B.blk_off) * kAtomBlock + (int)threadIdx.x;
  const bool active = local < B.n_atoms;
  const int64_t N = v.N;
  const int64_t i = (int64_t)B.atom_off + local;
  int c = 0;
  if (active) {
    double x = v.pos[i], y = v.pos[N + i], z = v.pos[2 * N + i];
    bool moved = false;
    if (KICK) {
      const Kick q = load_kick(v, b);
      const double h = kdt * ff.acc_over_m[v.type[i]];
      const double vx = q.post * (q.pre * (v.vel[i] - q.ux) + h * (double)f[i]);
      const double vy = q.post * (q.pre * (v.vel[N + i] - q.uy) + h * (double)f[N + i]);
      const double vz = q.post * (q.pre * (v.vel[2 * N + i] - q.uz) + h * (double)f[2 * N + i]);
      v.vel[i] = vx;
      v.vel[N + i] = vy;
      v.vel[2 * N + i] = vz;
      x += dt * vx;
      y += dt * vy;
      z += dt * vz;
      moved = true;
    }
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      atomicOr(v.err, (int)kErrNonFinite);
      x = y = z = 0.0;   // keep every index in range; the run is already invalid
      moved = true;
    }
    const double wx = wrap_coord(x, B.L[0], B.invL[0]);
    const double wy = wrap_coord(y, B.L[1], B.invL[1]);
    const double wz = wrap_coord(z, B.L[2], B.invL[2]);
    if (moved || wx != x || wy != y || wz != z) {
      v.pos[i] = wx;
      v.pos[N + i] = wy;
      v.pos[2 * N + i] = wz;
    }
    const int kx = cell_coord(wx, B.cinv[0], B.M[0]);
    const int ky = cell_coord(wy, B.cinv[1], B.M[1]);
    const int kz = cell_coord(wz, B.cinv[2], B.M[2]);
    c = B.cell_off + kx + B.M[0] * (ky + B.M[1] * kz);
    v.cell[i] = c;
  }
  const int s = aggregated_slot(v.cnt, c, active);
  if (active) v.slot[i] = s;
}

// ---- exclusive scan of the counts ----
template <typename T>
__device__ T block_exclusive_scan(T val, T* sh, T* total) {
  const int ln = lane(), w = (int)threadIdx.x >> 6;
  const int nw = (int)blockDim.x >> 6;
  T inc = val;
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(inc, d, 64);
    if (ln >= d) inc += t;
  }
  if (ln == 63) sh[w] = inc;
  __syncthreads();
  if (w == 0) {
    T x = ln < nw ? sh[ln] : 0;
    T xi = x;
    for (int d = 1; d < 64; d <<= 1) {
      T t = __shfl_up(xi, d, 64);
      if (ln >= d) xi += t;
    }
    if (ln < nw) sh[ln] = xi - x;
    if (ln == nw - 1) sh[32] = xi;
  }
  __syncthreads();
  const T ex = sh[w] + inc - val;
  *total = sh[32];
  __syncthreads();
  return ex;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const int32_t* __restrict__ cnt, int64_t C,
                                                          int32_t* tiles, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int sh[33];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < C) s += cnt[base + k];
  int total;
  block_exclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

// Tile b's offset is the sum of the tile totals tiles[0..b) (each block sums them itself: no
// separate pass over the tile totals), then the tile's own counts are scanned (k_scatter
// clears them for the next binning).  ONE (grids of at most kScanOnePass tiles): no tile
// totals; block b sums the counts of tiles 0..b-1 itself (all full tiles: each thread reads
// its four counts of each, the reads in flight together), one launch instead of two.
template <bool ONE>
__global__ __launch_bounds__(kScanBlock) void k_scan(int32_t* __restrict__ cnt, int64_t C,
                                                    const int32_t* __restrict__ tiles,
                                                    int32_t* __restrict__ cell_start,
                                                    const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ long long sh[33];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int vals[kScanItems];
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = base + k < C ? cnt[base + k] : 0;
    s += vals[k];
  }
  int pre = 0;
  if constexpr (ONE) {
    // all reads issued at once: tile min(t, b - 1) (in range), counted for t < b only
    const int4* __restrict__ c4 = reinterpret_cast<const int4*>(cnt);
    const int nb = (int)blockIdx.x;
    if (nb > 0) {
      int4 q[kScanOnePass - 1];
#pragma unroll
      for (int t = 0; t < kScanOnePass - 1; ++t) q[t] = c4[min(t, nb - 1) * (kScanTile / 4) + (int)threadIdx.x];
#pragma unroll
      for (int t = 0; t < kScanOnePass - 1; ++t) pre += t < nb ? (q[t].x + q[t].y) + (q[t].z + q[t].w) : 0;
    }
  } else {
    for (int t = (int)threadIdx.x; t < (int)blockIdx.x; t += kScanBlock) pre += tiles[t];
  }
  // one block scan of pre << 32 | s: the high half totals to the tile's offset and the low
  // half scans the tile's counts (both below 2^31, so no carry crosses the halves)
  long long tot2;
  const long long ex2 = block_exclusive_scan(((long long)pre << 32) | (long long)s, sh, &tot2);
  const int offset = (int)(tot2 >> 32), total = (int)(tot2 & 0xffffffffll);
  int ex = (int)(ex2 & 0xffffffffll) + offset;
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < C) cell_start[base + k] = ex;
    ex += vals[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) cell_start[C] = offset + total;
}

__global__ __launch_bounds__(kAtomBlock) void k_scatter(Views v, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int local = ((int)blockIdx.x - B.blk_off) * kAtomBlock + (int)threadIdx.x;
  const bool active = local < B.n_atoms;
  const int64_t i = (int64_t)B.atom_off + local;
  int32_t c = 0, sl = 0;
  if (active) {
    c = v.cell[i];
    sl = v.slot[i];
  }
  // the scan has read the counts: clear them for the next binning
  for (int64_t k = (int64_t)blockIdx.x * kAtomBlock + threadIdx.x; k < v.C; k += (int64_t)gridDim.x * kAtomBlock)
    v.cnt[k] = 0;
  if (active) v.tmp[v.cell_start[c] + sl] = (int32_t)i;
}

template <typename PayT>
__device__ inline void store_payload(PayT* p, int64_t dst, double rx, double ry, double rz, int32_t tag);

template <>
__device__ inline void store_payload<int4>(int4* p, int64_t dst, double rx, double ry, double rz,
                                           int32_t tag) {
  p[dst] = make_int4((int)rint(rx * kFix), (int)rint(ry * kFix), (int)rint(rz * kFix), tag);
}
template <>
__device__ inline void store_payload<Pay64>(Pay64* p, int64_t dst, double rx, double ry, double rz,
                                            int32_t tag) {
  Pay64 q;
  q.x = rx;
  q.y = ry;
  q.z = rz;
  q.tagbits = __longlong_as_double((long long)tag);
  p[dst] = q;
}

constexpr int kRankBatch = 4;   // list entries read together by the rank walk

template <typename PayT>
__global__ __launch_bounds__(kAtomBlock) void k_rank_payload(Views v, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int local = ((int)blockIdx.x - B.blk_off) * kAtomBlock + (int)threadIdx.x;
  if (local >= B.n_atoms) return;
  const int64_t N = v.N;
  const int32_t i = B.atom_off + local;
  // the loads that depend on i alone go first, so they are in flight during the rank walk
  const double x = v.pos[i], y = v.pos[N + i], z = v.pos[2 * N + i];
  const int32_t ty = v.type[i];
  const int32_t c = v.cell[i];
  const int32_t s0 = v.cell_start[c];
  const int32_t n = v.cell_start[c + 1] - s0;
  // the unordered list in batches of kRankBatch entries whose loads are in flight together;
  // entries past the end re-read the last one (atom i is in the cell, so n >= 1) and count 0
  int rank = 0;
  for (int k0 = 0; k0 < n; k0 += kRankBatch) {
    int32_t t[kRankBatch];
#pragma unroll
    for (int u = 0; u < kRankBatch; ++u) t[u] = v.tmp[s0 + min(k0 + u, n - 1)];
#pragma unroll
    for (int u = 0; u < kRankBatch; ++u) rank += (k0 + u < n && t[u] < i) ? 1 : 0;
  }
  if (rank >= n) rank = n - 1;   // only reachable if the lists were inconsistent
  const int32_t dst = s0 + rank;
  v.cell_atoms[dst] = i;
  v.scell[dst] = c;
  const int kx = cell_coord(x, B.cinv[0], B.M[0]);
  const int ky = cell_coord(y, B.cinv[1], B.M[1]);
  const int kz = cell_coord(z, B.cinv[2], B.M[2]);
  const double rx = x - ((double)kx + 0.5) * B.edge[0];
  const double ry = y - ((double)ky + 0.5) * B.edge[1];
  const double rz = z - ((double)kz + 0.5) * B.edge[2];
  const int32_t tag = (i << 4) | ((ty & 1) << 3) | (kx & 7);
  store_payload<PayT>(static_cast<PayT*>(v.payload), dst, rx, ry, rz, tag);
  if (v.nl_cap) {   // neighbour-list mode: where the list build saw the atom; the current payload
    store_payload<PayT>(static_cast<PayT*>(v.pay_cur), dst, rx, ry, rz, tag);   // is the build's
    v.slot_of[i] = dst;
    v.x_build[i] = x;
    v.x_build[N + i] = y;
    v.x_build[2 * N + i] = z;
  }
}

// ---- neighbour-list mode: the update between list builds ----
__device__ inline double min_image(double d, double L, double invL) { return d - L * rint(d * invL); }

template <typename PayT>
__device__ inline void refresh_payload(const PayT* build, PayT* cur, int32_t s, double dx, double dy, double dz);

template <>
__device__ inline void refresh_payload<int4>(const int4* build, int4* cur, int32_t s, double dx, double dy,
                                             double dz) {
  const int4 q = build[s];
  cur[s] = make_int4(q.x + (int)rint(dx * kFix), q.y + (int)rint(dy * kFix), q.z + (int)rint(dz * kFix), q.w);
}
template <>
__device__ inline void refresh_payload<Pay64>(const Pay64* build, Pay64* cur, int32_t s, double dx, double dy,
                                              double dz) {
  Pay64 q = build[s];
  q.x += dx;
  q.y += dy;
  q.z += dz;
  cur[s] = q;
}

// Velocity update, drift and wrap as in k_bin_count, without binning; then
// the displacement since the list build moves the atom's build payload to its current place:
// cur = build + round(d * 2^25) (mixed) or build + d (FP64), so pair differences stay exact
// integers in the mixed form.  A displacement above half the skin (or force) raises the
// rebuild flag: this step's gated bin and list kernels then rebuild from the new positions
// before the forces are evaluated, so the list in use always holds every pair within rc.
template <typename F, typename PayT>
__global__ __launch_bounds__(kAtomBlock) void k_nl_integrate(Views v, const F* __restrict__ f, double dt,
                                                          double kdt, FFDev ff, int force) {
  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int local = ((int)blockIdx.x - B.blk_off) * kAtomBlock + (int)threadIdx.x;
  if (force && blockIdx.x == 0 && threadIdx.x == 0) *v.nl_flag = 1;
  if (local >= B.n_atoms) return;
  const int64_t N = v.N;
  const int64_t i = (int64_t)B.atom_off + local;
  const Kick q = load_kick(v, b);
  const double h = kdt * ff.acc_over_m[v.type[i]];
  const double vx = q.post * (q.pre * (v.vel[i] - q.ux) + h * (double)f[i]);
  const double vy = q.post * (q.pre * (v.vel[N + i] - q.uy) + h * (double)f[N + i]);
  const double vz = q.post * (q.pre * (v.vel[2 * N + i] - q.uz) + h * (double)f[2 * N + i]);
  v.vel[i] = vx;
  v.vel[N + i] = vy;
  v.vel[2 * N + i] = vz;
  double x = v.pos[i] + dt * vx, y = v.pos[N + i] + dt * vy, z = v.pos[2 * N + i] + dt * vz;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    atomicOr(v.err, (int)kErrNonFinite);
    x = y = z = 0.0;
  }
  x = wrap_coord(x, B.L[0], B.invL[0]);
  y = wrap_coord(y, B.L[1], B.invL[1]);
  z = wrap_coord(z, B.L[2], B.invL[2]);
  v.pos[i] = x;
  v.pos[N + i] = y;
  v.pos[2 * N + i] = z;
  const double dx = min_image(x - v.x_build[i], B.L[0], B.invL[0]);
  const double dy = min_image(y - v.x_build[N + i], B.L[1], B.invL[1]);
  const double dz = min_image(z - v.x_build[2 * N + i], B.L[2], B.invL[2]);
  const bool moved = dx * dx + dy * dy + dz * dz > v.nl_half_skin2;
  if (__builtin_amdgcn_ballot_w64(moved) != 0 && lane() == 0) *v.nl_flag = 1;   // same value from every writer
  refresh_payload<PayT>(static_cast<const PayT*>(v.payload), static_cast<PayT*>(v.pay_cur), v.slot_of[i], dx, dy,
                        dz);
}

// ---- bonded terms ----
template <typename P>
struct V3 {
  P x, y, z;
};
template <typename P>
__device__ inline V3<P> v3(P x, P y, P z) {
  return V3<P>{x, y, z};
}
template <typename P>
__device__ inline P dot(V3<P> a, V3<P> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename P>
__device__ inline V3<P> cross(V3<P> a, V3<P> b) {
  return V3<P>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename P>
__device__ inline V3<P> scale(V3<P> a, P s) {
  return V3<P>{a.x * s, a.y * s, a.z * s};
}
template <typename P>
__device__ inline V3<P> add(V3<P> a, V3<P> b) {
  return V3<P>{a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename P>
__device__ inline V3<P> neg(V3<P> a) {
  return V3<P>{-a.x, -a.y, -a.z};
}

__device__ inline double sqrt_p(double x) { return sqrt(x); }
__device__ inline float sqrt_p(float x) { return sqrtf(x); }
__device__ inline double atan2_p(double y, double x) { return atan2(y, x); }
__device__ inline float atan2_p(float y, float x) { return atan2f(y, x); }

// Minimum-image difference b - a along one dimension, in FP64, then cast.
template <typename P>
__device__ inline V3<P> mi_diff(const double* xs, int a, int b, int stride, const BoxDev& B) {
  double d[3];
  for (int k = 0; k < 3; ++k) {
    double t = xs[k * stride + b] - xs[k * stride + a];
    d[k] = t - B.L[k] * rint(t * B.invL[k]);
  }
  return v3<P>((P)d[0], (P)d[1], (P)d[2]);
}

// The bonded kernel runs kAtomBlock atoms per work-group.  The mixed form runs it on one more
// wavefront than it has atoms: the 3 term starts and 6 staged positions beyond the first
// kAtomBlock go to that wave instead of a second pass of wave 0 (it owns no atom; its partial
// sums are exact zeros).  The FP64 form, whose LDS arrays allow 3 work-groups per CU, measured
// faster without it.
constexpr int kBondedThreads = kAtomBlock + 64;
template <typename P>
constexpr int bonded_threads() { return std::is_same<P, double>::value ? kAtomBlock : kBondedThreads; }

// MODE (BondedMode): forces only, or also the second velocity-Verlet half kick, or (leap-frog)
// the kinetic energy of the velocities as they stand.  COM: also the box momentum partials.
template <typename P, int MODE, bool ENERGY, bool COM>
__global__ __launch_bounds__(bonded_threads<P>()) void k_bonded(Views v, FFDev ff, double dt) {
  constexpr bool KICK = MODE == kBondedVerletKick;
  constexpr bool SUMS = MODE != kBondedForces || ENERGY;   // block partials written
  constexpr int NP = COM ? 8 : 5;
  static_assert(NP <= kBdParts, "partials");
  constexpr int S = kAtomBlock + 2 * kHalo;       // staged atoms: [g0 - 3, g0 + 256 + 3)
  constexpr int T = kAtomBlock + kHalo;           // term starts:  [g0 - 3, g0 + 256)
  __shared__ double xs[3 * S];
  // per term start u: bond force on its first atom; angle forces on i and k;
  // dihedral forces on i, j and l (the missing atom gets minus the sum)
  __shared__ P fb[3 * T], fai[3 * T], fak[3 * T], fdi[3 * T], fdj[3 * T], fdl[3 * T];
  constexpr int NT = bonded_threads<P>();
  __shared__ dd red[NT / 64][NP];

  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int64_t N = v.N;
  const int32_t g0 = B.atom_off + ((int)blockIdx.x - B.blk_off) * kAtomBlock;
  const int32_t box_end = B.atom_off + B.n_atoms;
  const int L = ff.chain_len;

  for (int t = threadIdx.x; t < S; t += NT) {
    const int32_t g = g0 - kHalo + t;
    const bool ok = g >= B.atom_off && g < box_end;
    xs[t] = ok ? v.pos[g] : 0.0;
    xs[S + t] = ok ? v.pos[N + g] : 0.0;
    xs[2 * S + t] = ok ? v.pos[2 * N + g] : 0.0;
  }
  __syncthreads();

  double e_b = 0.0, e_a = 0.0, e_d = 0.0, w_b = 0.0;
  const P kb = (P)ff.kb, ka = (P)ff.ka, kphi = (P)ff.kphi;
  for (int u = threadIdx.x; u < T; u += NT) {
    const int32_t p = g0 - kHalo + u;   // first atom of the terms starting here
    const bool in_box = p >= B.atom_off && p < box_end;
    const int q = in_box ? (int)((p - B.atom_off) % L) : L;   // site within the chain
    const bool own = ENERGY && p >= g0 && p < g0 + kAtomBlock && in_box;
    V3<P> zero = v3<P>(0, 0, 0);
    // the chain's bond vectors from p, each computed once: b1 = x_{p+1} - x_p,
    // b2 = x_{p+2} - x_{p+1}, b3 = x_{p+3} - x_{p+2}; a difference taken the other way is the
    // exact negation (subtraction, rint and the fused multiply-add are all odd in the difference)
    V3<P> b1 = zero, b2 = zero, b3 = zero;
    if (q + 1 < L) b1 = mi_diff<P>(xs, u, u + 1, S, B);
    if (q + 2 < L) b2 = mi_diff<P>(xs, u + 1, u + 2, S, B);
    if (q + 3 < L) b3 = mi_diff<P>(xs, u + 2, u + 3, S, B);
    // bond (p, p+1), Eq. (4)
    V3<P> f_b = zero;
    if (q + 1 < L) {
      const V3<P> d = b1;                                    // x_{p+1} - x_p
      const double d2 = (double)dot(d, d);
      const double r = sqrt(d2);
      const P dr = (P)(r - ff.b0);
      f_b = scale(d, kb * dr / (P)r);                        // force on p
      if (own) {
        e_b += 0.5 * ff.kb * (double)dr * (double)dr;
        w_b += (double)dot(d, neg(f_b));                     // (x_{p+1} - x_p) . F_{p+1}
      }
    }
    // angle (p, p+1, p+2) at p+1, Eq. (5)
    V3<P> f_ai = zero, f_ak = zero;
    if (q + 2 < L) {
      const V3<P> a = neg(b1);                               // x_i - x_j
      const V3<P> c = b2;                                    // x_k - x_j
      const P ac = dot(a, c), aa = dot(a, a), cc = dot(c, c);
      const V3<P> axc = cross(a, c);
      const P s = sqrt_p(dot(axc, axc));                     // |a||c| sin(theta)
      const P th = atan2_p(s, ac);
      const P dth = (P)((double)th - ff.theta0);
      const P g = ka * dth / s;
      f_ai = scale(add(c, scale(a, -ac / aa)), g);
      f_ak = scale(add(a, scale(c, -ac / cc)), g);
      if (own) {
        e_a += 0.5 * ff.ka * (double)dth * (double)dth;
        w_b += (double)(dot(a, f_ai) + dot(c, f_ak));
      }
    }
    // dihedral (p, p+1, p+2, p+3), Eq. (6), IUPAC angle
    V3<P> f_di = zero, f_dj = zero, f_dl = zero;
    if (q + 3 < L) {
      const V3<P> rij = neg(b1);                               // x_i - x_j
      const V3<P> rkj = b2;                                    // x_k - x_j
      const V3<P> rkl = neg(b3);                               // x_k - x_l
      const V3<P> m = cross(rij, rkj);
      const V3<P> n = cross(rkj, rkl);
      const P mm = dot(m, m), nn = dot(n, n), kk = dot(rkj, rkj);
      const P lk = sqrt_p(kk);
      const P craw = dot(m, n);
      const P sraw = lk * dot(rij, n);
      const P rho = sqrt_p(craw * craw + sraw * sraw);      // |m||n|
      const P cphi = craw / rho, sphi = sraw / rho;
      // cos(n phi), sin(n phi) by the angle-addition recurrence
      P cn = cphi, sn = sphi;
      for (int t = 1; t < ff.n_dih; ++t) {
        const P c2 = cn * cphi - sn * sphi;
        sn = sn * cphi + cn * sphi;
        cn = c2;
      }
      const P cps = (P)ff.cos_phis, sps = (P)ff.sin_phis;
      // E = kphi (1 + cos(n phi - phis)); dE/dphi = -n kphi sin(n phi - phis)
      const P dEdphi = -(P)ff.n_dih * kphi * (sn * cps - cn * sps);
      const V3<P> dpi = scale(m, lk / mm);                   // d phi / d x_i
      const V3<P> dpl = scale(n, -lk / nn);                  // d phi / d x_l
      const P pp = dot(rij, rkj) / kk, qq = dot(rkl, rkj) / kk;
      const V3<P> dpj = add(scale(dpi, pp - (P)1), scale(dpl, -qq));
      f_di = scale(dpi, -dEdphi);
      f_dj = scale(dpj, -dEdphi);
      f_dl = scale(dpl, -dEdphi);
      if (own) {
        e_d += (double)(kphi * ((P)1 + (cn * cps + sn * sps)));
        // (x_i - x_j).F_i + (x_k - x_j).F_k + (x_l - x_j).F_l with F_k = -(F_i + F_j + F_l)
        const V3<P> f_dk = neg(add(add(f_di, f_dj), f_dl));
        const V3<P> rlj = add(rkj, neg(rkl));                // x_l - x_j
        w_b += (double)(dot(rij, f_di) + dot(rkj, f_dk) + dot(rlj, f_dl));
      }
    }
    fb[3 * u] = f_b.x; fb[3 * u + 1] = f_b.y; fb[3 * u + 2] = f_b.z;
    fai[3 * u] = f_ai.x; fai[3 * u + 1] = f_ai.y; fai[3 * u + 2] = f_ai.z;
    fak[3 * u] = f_ak.x; fak[3 * u + 1] = f_ak.y; fak[3 * u + 2] = f_ak.z;
    fdi[3 * u] = f_di.x; fdi[3 * u + 1] = f_di.y; fdi[3 * u + 2] = f_di.z;
    fdj[3 * u] = f_dj.x; fdj[3 * u + 1] = f_dj.y; fdj[3 * u + 2] = f_dj.z;
    fdl[3 * u] = f_dl.x; fdl[3 * u + 1] = f_dl.y; fdl[3 * u + 2] = f_dl.z;
  }
  __syncthreads();

  const int t = threadIdx.x;
  const int32_t g = g0 + t;
  double ke = 0.0, mom[3] = {0.0, 0.0, 0.0};
  if (t < kAtomBlock && g < box_end) {
    const int u = t + kHalo;   // term start index of the terms that begin at atom g
    P f[3];
    for (int k = 0; k < 3; ++k) {
      // fixed order: dihedrals (g as l, k, j, i), angles (k, j, i), bonds (second, first)
      P s = fdl[3 * (u - 3) + k];
      s += -(fdi[3 * (u - 2) + k] + fdj[3 * (u - 2) + k] + fdl[3 * (u - 2) + k]);
      s += fdj[3 * (u - 1) + k];
      s += fdi[3 * u + k];
      s += fak[3 * (u - 2) + k];
      s += -(fai[3 * (u - 1) + k] + fak[3 * (u - 1) + k]);
      s += fai[3 * u + k];
      s += -fb[3 * (u - 1) + k];
      s += fb[3 * u + k];
      f[k] = s;
    }
    const P* flj = static_cast<const P*>(v.f_lj);
    P* ftot = static_cast<P*>(v.f_tot);
    for (int k = 0; k < 3; ++k) {
      f[k] += flj[k * N + g];
      ftot[k * N + g] = f[k];
    }
    if (SUMS) {
      const int ty = v.type[g];
      double vv[3];
      for (int k = 0; k < 3; ++k) vv[k] = v.vel[k * N + g];
      if (KICK) {
        const double h = 0.5 * dt * ff.acc_over_m[ty];
        for (int k = 0; k < 3; ++k) {
          vv[k] += h * (double)f[k];
          v.vel[k * N + g] = vv[k];
        }
      }
      ke = ff.half_m_over_acc[ty] * (vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
      if (COM)
        for (int k = 0; k < 3; ++k) mom[k] = ff.mass[ty] * vv[k];
    }
  }
  if (SUMS) {
    // block partials: E_b, E_a, E_d, W_b, KE [, momentum xyz] (double-double, fixed order)
    dd q[NP];
    q[0] = dd_from(e_b);
    q[1] = dd_from(e_a);
    q[2] = dd_from(e_d);
    q[3] = dd_from(w_b);
    q[4] = dd_from(ke);
    if (COM)
      for (int k = 0; k < 3; ++k) q[5 + k] = dd_from(mom[k]);
    for (int k = 0; k < NP; ++k)
      for (int off = 32; off > 0; off >>= 1) {
        dd o{__shfl_xor(q[k].hi, off), __shfl_xor(q[k].lo, off)};
        q[k] = dd_add(q[k], o);
      }
    if (lane() == 0)
      for (int k = 0; k < NP; ++k) red[threadIdx.x >> 6][k] = q[k];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < NP; ++k) {
        dd s = red[0][k];
        for (int w = 1; w < NT / 64; ++w) s = dd_add(s, red[w][k]);
        v.part_bd[(int64_t)k * v.n_atom_blocks + blockIdx.x] = s;
      }
  }
}

// Sums NV double-double values over the block in a fixed order (each thread's own values,
// then a butterfly over the wave, then the waves in order); every thread gets the sums.
template <int NV>
__device__ void block_sums(dd (&s)[NV], dd (*sh)[NV]) {
  for (int k = 0; k < NV; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      dd o{__shfl_xor(s[k].hi, off), __shfl_xor(s[k].lo, off)};
      s[k] = dd_add(s[k], o);
    }
  if (lane() == 0)
    for (int k = 0; k < NV; ++k) sh[threadIdx.x >> 6][k] = s[k];
  __syncthreads();
  for (int k = 0; k < NV; ++k) {
    dd r = sh[0][k];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = dd_add(r, sh[w][k]);
    s[k] = r;
  }
  __syncthreads();
}

// First level of the per-box reduction for large boxes: block g sums one chunk of at most
// kReduceChunk block partials (chunks [0, n_bd_chunks) hold bonded/kinetic partials, the rest
// LJ partials), thread t adding partials t, t + 256, ... of the chunk in that order with their
// loads in flight together, then the block in a fixed order.  The bonded sums are stored in
// k_reduce's order (KE, [momentum xyz], [E_b E_a E_d W_b]), the LJ sums as E, E_shifted, W.
template <bool ENERGY, bool COM>
__global__ __launch_bounds__(256) void k_reduce_l1(Views v, int first_chunk) {
  constexpr int iP = 1, iE = COM ? 4 : 1, NB = iE + (ENERGY ? 4 : 0);
  constexpr int NQ = NB > 3 ? NB : 3;
  constexpr int kPer = kReduceChunk / 256;
  __shared__ dd sh[4][NQ];
  const int g = first_chunk + (int)blockIdx.x;
  const int2 rng = v.chunk_rng[g];
  const bool bonded = g < v.n_bd_chunks;
  dd q[NQ];
  for (int k = 0; k < NQ; ++k) q[k] = dd{0.0, 0.0};
  dd r[kPer][NQ];
  const int64_t nb = v.n_atom_blocks;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int j = min(rng.x + (int)threadIdx.x + 256 * u, rng.y - 1);   // past the end: re-read, not added
    if (bonded) {
      const dd* p = v.part_bd + j;
      r[u][0] = p[4 * nb];
      if (COM)
        for (int k = 0; k < 3; ++k) r[u][iP + k] = p[(5 + k) * nb];
      if (ENERGY)
        for (int k = 0; k < 4; ++k) r[u][iE + k] = p[k * nb];
    } else {
      for (int k = 0; k < 3; ++k) r[u][k] = v.part_lj[(int64_t)j * 3 + k];
    }
  }
  const int nq = bonded ? NB : 3;
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (rng.x + (int)threadIdx.x + 256 * u < rng.y)
      for (int k = 0; k < nq; ++k) q[k] = dd_add(q[k], r[u][k]);
  block_sums<NQ>(q, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < nq; ++k) v.part_l1[(int64_t)g * kBdParts + k] = q[k];
}

// One block per box: the box's energies, kinetic energy and temperature, all partials read
// in one pass (for large boxes, the first level's chunk sums, l1_bd / l1_lj); with update,
// the integrator state the next step applies:
//   velocity Verlet: the Berendsen factor lambda = sqrt(1 + dt/tau (T0/T - 1));
//   leap-frog: xi' = xi + dt omega^2 (T/T0 - 1), omega = 2 pi / tau, eta += dt (xi + xi')/2,
//              and the kick factors 1 - dt xi'/2 and 1 / (1 + dt xi'/2);
//   COM removal: u = P / M, and the kinetic energy of the motion relative to it,
//              KE - |P|^2 / (2 M).
// Bonded partials: 0 E_b, 1 E_a, 2 E_d, 3 W_b, 4 KE, 5..7 momentum; LJ: E, E_shifted, W.
// ENERGY: the energies and virial too; COM (with update): the momentum and u.
// Neighbour-list mode, with update: the step's rebuild flag has been read by every kernel
// that uses it, so it is counted and cleared here for the next step.
template <bool ENERGY, bool COM>
__global__ __launch_bounds__(256) void k_reduce(Views v, int update, StepOpts o, int l1_bd, int l1_lj) {
  // q: KE, [momentum xyz], [E_b E_a E_d W_b E_lj E_lj_shifted W_lj]
  constexpr int iP = 1, iE = COM ? 4 : 1, NV = iE + (ENERGY ? 7 : 0);
  __shared__ dd sh[4][NV];
  const int b = blockIdx.x;
  if (update && v.nl_flag && b == 0 && threadIdx.x == 0 && *v.nl_flag) {
    *v.nl_builds += 1ull;
    *v.nl_flag = 0;
  }
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int first = B.blk_off;
  const int count = (B.n_atoms + kAtomBlock - 1) / kAtomBlock;
  dd q[NV];
  for (int k = 0; k < NV; ++k) q[k] = dd{0.0, 0.0};
  // thread t adds partials t, t + 256, t + 512, ... in that order; the loads of kBatch of them
  // are issued together (a partial past the end re-reads the last one and is not added), so
  // a large box (117k partials at 30M atoms) waits for one round trip per batch, not per partial
  constexpr int NB = iE + (ENERGY ? 4 : 0);   // bonded partials read per work-group
  constexpr int kBatch = NB <= 4 ? 8 : 4;
  if (l1_bd) {
    for (int t = threadIdx.x; t < B.bd_chunks; t += blockDim.x)
      for (int k = 0; k < NB; ++k) q[k] = dd_add(q[k], v.part_l1[(int64_t)(B.bd_chunk_off + t) * kBdParts + k]);
  }
  for (int t0 = threadIdx.x; !l1_bd && t0 < count; t0 += blockDim.x * kBatch) {
    dd r[kBatch][NB];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // partial k of block j at part_bd[k * n_atom_blocks + j]: consecutive lanes, consecutive blocks
      const dd* p = v.part_bd + first + min(t0 + u * (int)blockDim.x, count - 1);
      const int64_t nb = v.n_atom_blocks;
      r[u][0] = p[4 * nb];
      if (COM)
        for (int k = 0; k < 3; ++k) r[u][iP + k] = p[(5 + k) * nb];
      if (ENERGY)
        for (int k = 0; k < 4; ++k) r[u][iE + k] = p[k * nb];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (t0 + u * (int)blockDim.x < count)
        for (int k = 0; k < NB; ++k) q[k] = dd_add(q[k], r[u][k]);
  }
  if (ENERGY) {
    if (l1_lj) {
      for (int t = threadIdx.x; t < B.lj_chunks; t += blockDim.x)
        for (int k = 0; k < 3; ++k)
          q[iE + 4 + k] = dd_add(q[iE + 4 + k], v.part_l1[(int64_t)(B.lj_chunk_off + t) * kBdParts + k]);
    } else {
      const int lfirst = B.lj_blk_off;
      const int lcount = (b + 1 < v.n_boxes ? v.boxes[b + 1].lj_blk_off : v.n_lj_blocks) - lfirst;
      for (int t = threadIdx.x; t < lcount; t += blockDim.x)
        for (int k = 0; k < 3; ++k) q[iE + 4 + k] = dd_add(q[iE + 4 + k], v.part_lj[(int64_t)(lfirst + t) * 3 + k]);
    }
  }
  block_sums<NV>(q, sh);
  double KE = q[0].hi + q[0].lo;
  double u[3] = {0.0, 0.0, 0.0};
  if (COM) {
    double p[3];
    for (int k = 0; k < 3; ++k) {
      p[k] = q[iP + k].hi + q[iP + k].lo;
      u[k] = p[k] * B.inv_mass;
    }
    KE -= 0.5 * (p[0] * u[0] + p[1] * u[1] + p[2] * u[2]) / kAccUnit;
  }
  const double T = 2.0 * KE / (B.dof * kRgas);
  double* out = v.energy + (int64_t)b * kEnergySlots;
  if (threadIdx.x != 0) return;
  if (ENERGY) {
    out[0] = q[iE + 4].hi + q[iE + 4].lo;
    out[1] = q[iE + 5].hi + q[iE + 5].lo;
    out[2] = q[iE].hi + q[iE].lo;
    out[3] = q[iE + 1].hi + q[iE + 1].lo;
    out[4] = q[iE + 2].hi + q[iE + 2].lo;
    const dd w = dd_add(q[iE + 6], q[iE + 3]);
    out[7] = w.hi + w.lo;
  }
  out[5] = KE;
  out[6] = T;
  double* th = v.thermo + (int64_t)b * kThermo;
  const double two_pi = 6.283185307179586;
  const double w2 = (two_pi / o.tau) * (two_pi / o.tau);
  const bool lf = o.integrator == kLeapfrogNoseHoover;
  if (update) {
    if (!lf) {
      double lam = 1.0;
      if (B.T0 > 0.0 && T > 0.0) lam = sqrt(1.0 + o.dt / o.tau * (B.T0 / T - 1.0));
      th[kThPre] = lam;
    } else if (B.T0 > 0.0) {
      const double xi = th[kThXi];
      const double xn = xi + o.dt * w2 * (T / B.T0 - 1.0);
      th[kThEta] += 0.5 * o.dt * (xi + xn);
      th[kThXi] = xn;
      th[kThPre] = 1.0 - 0.5 * o.dt * xn;
      th[kThPost] = 1.0 / (1.0 + 0.5 * o.dt * xn);
    }
    if (COM)
      for (int k = 0; k < 3; ++k) th[kThU + k] = u[k];
  }
  const double xi = th[kThXi];
  out[8] = xi;
  out[9] = lf && B.T0 > 0.0 ? B.dof * kRgas * B.T0 * (xi * xi / (2.0 * w2) + th[kThEta]) : 0.0;
}

// Applies the pending Berendsen factor (velocity Verlet) and COM velocity to v.
__global__ __launch_bounds__(kAtomBlock) void k_finalize(Views v, int lf) {
  const int b = v.blk_box[blockIdx.x];
  const BoxDev B = v.boxes[b];   // read at entry, before any store: scalar loads
  const int local = ((int)blockIdx.x - B.blk_off) * kAtomBlock + (int)threadIdx.x;
  if (local >= B.n_atoms) return;
  const int64_t N = v.N;
  const int64_t i = (int64_t)B.atom_off + local;
  const double* th = v.thermo + (int64_t)b * kThermo;
  const double s = lf ? 1.0 : th[kThPre];
  v.vel[i] = s * (v.vel[i] - th[kThU]);
  v.vel[N + i] = s * (v.vel[N + i] - th[kThU + 1]);
  v.vel[2 * N + i] = s * (v.vel[2 * N + i] - th[kThU + 2]);
}

// After k_finalize: nothing pending (the leap-frog kick factors are state, not pending).
__global__ void k_clear_pending(double* thermo, int n_boxes, int lf) {
  for (int b = (int)threadIdx.x; b < n_boxes; b += (int)blockDim.x) {
    double* th = thermo + (int64_t)b * kThermo;
    if (!lf) th[kThPre] = 1.0;
    th[kThU] = th[kThU + 1] = th[kThU + 2] = 0.0;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}
__global__ void k_fill_f64(double* p, int64_t n, double val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65535 * 8) g = 65535 * 8;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

static double kick_dt(const StepOpts& o) { return o.integrator == kLeapfrogNoseHoover ? o.dt : 0.5 * o.dt; }

void launch_bin_count(const Views& v, bool kick, const StepOpts& o, const FFDev& ff, bool fp32_force,
                      hipStream_t s, const int32_t* gate) {
  dim3 g(v.n_atom_blocks), blk(kAtomBlock);
  const double kdt = kick_dt(o);
  if (!kick)
    hipLaunchKernelGGL((k_bin_count<float, false>), g, blk, 0, s, v, (const float*)nullptr, o.dt, kdt, ff, gate);
  else if (fp32_force)
    hipLaunchKernelGGL((k_bin_count<float, true>), g, blk, 0, s, v, (const float*)v.f_tot, o.dt, kdt, ff, gate);
  else
    hipLaunchKernelGGL((k_bin_count<double, true>), g, blk, 0, s, v, (const double*)v.f_tot, o.dt, kdt, ff, gate);
}

static int scan_tiles(const Views& v) { return (int)((v.C + kScanTile - 1) / kScanTile); }

void launch_scan(const Views& v, hipStream_t s, const int32_t* gate) {
  const int n = scan_tiles(v);
  if (n <= kScanOnePass) {
    hipLaunchKernelGGL(k_scan<true>, dim3(n), dim3(kScanBlock), 0, s, v.cnt, v.C, v.scan_tiles, v.cell_start, gate);
    return;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(n), dim3(kScanBlock), 0, s, v.cnt, v.C, v.scan_tiles, gate);
  hipLaunchKernelGGL(k_scan<false>, dim3(n), dim3(kScanBlock), 0, s, v.cnt, v.C, v.scan_tiles, v.cell_start, gate);
}

void launch_scatter(const Views& v, hipStream_t s, const int32_t* gate) {
  hipLaunchKernelGGL(k_scatter, dim3(v.n_atom_blocks), dim3(kAtomBlock), 0, s, v, gate);
}

void launch_rank_payload(const Views& v, bool fp32, hipStream_t s, const int32_t* gate) {
  if (fp32)
    hipLaunchKernelGGL(k_rank_payload<int4>, dim3(v.n_atom_blocks), dim3(kAtomBlock), 0, s, v, gate);
  else
    hipLaunchKernelGGL(k_rank_payload<Pay64>, dim3(v.n_atom_blocks), dim3(kAtomBlock), 0, s, v, gate);
}

template <typename P>
void launch_bonded_p(const Views& v, const FFDev& ff, BondedMode mode, bool energy, bool com, double dt,
                     hipStream_t s) {
  dim3 g(v.n_atom_blocks);
#define MDK_BONDED(M, E, C) hipLaunchKernelGGL((k_bonded<P, M, E, C>), g, dim3(bonded_threads<P>()), 0, s, v, ff, dt)
  if (mode == kBondedForces) {
    if (energy) MDK_BONDED(kBondedForces, true, false); else MDK_BONDED(kBondedForces, false, false);
  } else if (mode == kBondedVerletKick) {
    if (com) { if (energy) MDK_BONDED(kBondedVerletKick, true, true); else MDK_BONDED(kBondedVerletKick, false, true); }
    else { if (energy) MDK_BONDED(kBondedVerletKick, true, false); else MDK_BONDED(kBondedVerletKick, false, false); }
  } else {
    if (com) { if (energy) MDK_BONDED(kBondedLeapfrog, true, true); else MDK_BONDED(kBondedLeapfrog, false, true); }
    else { if (energy) MDK_BONDED(kBondedLeapfrog, true, false); else MDK_BONDED(kBondedLeapfrog, false, false); }
  }
#undef MDK_BONDED
}

void launch_bonded(const Views& v, const FFDev& ff, bool fp32, BondedMode mode, bool energy, bool com,
                   double dt, hipStream_t s) {
  if (fp32)
    launch_bonded_p<float>(v, ff, mode, energy, com, dt, s);
  else
    launch_bonded_p<double>(v, ff, mode, energy, com, dt, s);
}

// Large boxes go through the first-level chunk sums: the bonded chunks when some box has more
// than kReduceChunk atom blocks, the LJ chunks (energy evaluations only) when some box has more
// than kReduceChunk LJ blocks.
void launch_reduce(const Views& v, bool energy, bool update, const StepOpts& o, hipStream_t s) {
  const int u = update ? 1 : 0;
  const bool com = update && o.remove_com;
  const int l1_bd = v.l1_bd, l1_lj = energy && v.l1_lj ? 1 : 0;
  if (l1_bd || l1_lj) {
    const int c0 = l1_bd ? 0 : v.n_bd_chunks;
    const int c1 = l1_lj ? v.n_bd_chunks + v.n_lj_chunks : v.n_bd_chunks;
    const dim3 g(c1 - c0), blk(256);
#define MDK_L1(E, C) hipLaunchKernelGGL((k_reduce_l1<E, C>), g, blk, 0, s, v, c0)
    if (energy) { if (com) MDK_L1(true, true); else MDK_L1(true, false); }
    else { if (com) MDK_L1(false, true); else MDK_L1(false, false); }
#undef MDK_L1
  }
  if (energy) {
    if (com) hipLaunchKernelGGL((k_reduce<true, true>), dim3(v.n_boxes), dim3(256), 0, s, v, u, o, l1_bd, l1_lj);
    else hipLaunchKernelGGL((k_reduce<true, false>), dim3(v.n_boxes), dim3(256), 0, s, v, u, o, l1_bd, l1_lj);
  } else {
    if (com) hipLaunchKernelGGL((k_reduce<false, true>), dim3(v.n_boxes), dim3(256), 0, s, v, u, o, l1_bd, l1_lj);
    else hipLaunchKernelGGL((k_reduce<false, false>), dim3(v.n_boxes), dim3(256), 0, s, v, u, o, l1_bd, l1_lj);
  }
}

void launch_nl_integrate(const Views& v, const StepOpts& o, const FFDev& ff, bool fp32_force, bool force_build,
                         hipStream_t s) {
  dim3 g(v.n_atom_blocks), blk(kAtomBlock);
  const double kdt = kick_dt(o);
  const int fb = force_build ? 1 : 0;
  if (fp32_force)
    hipLaunchKernelGGL((k_nl_integrate<float, int4>), g, blk, 0, s, v, (const float*)v.f_tot, o.dt, kdt, ff, fb);
  else
    hipLaunchKernelGGL((k_nl_integrate<double, Pay64>), g, blk, 0, s, v, (const double*)v.f_tot, o.dt, kdt, ff, fb);
}

void launch_finalize(const Views& v, const StepOpts& o, hipStream_t s) {
  const int lf = o.integrator == kLeapfrogNoseHoover ? 1 : 0;
  hipLaunchKernelGGL(k_finalize, dim3(v.n_atom_blocks), dim3(kAtomBlock), 0, s, v, lf);
  hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(64), 0, s, v.thermo, v.n_boxes, lf);
}

}  // namespace mdk
