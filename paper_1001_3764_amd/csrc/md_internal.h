// Internal declarations of the gfx950 MD library (device structs, launchers).
// Not part of the C ABI; see include/md.h for the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mdk {

constexpr int kAtomBlock = 256;   // threads per block of every per-atom kernel
constexpr int kLjAtomBlock = 128; // threads per block of the lane-per-atom LJ kernel
constexpr int kScanItems = 4;     // cells per thread in the scan
constexpr int kScanBlock = 1024;
constexpr int kScanTile = kScanItems * kScanBlock;
constexpr int kScanOnePass = 16;  // at most this many tiles: the one-launch scan
constexpr int kHalo = 3;          // a dihedral reaches 3 atoms beyond its first atom

// acceleration of 1 kcal/mol/A on 1 g/mol, in A/fs^2; gas constant in kcal/mol/K
constexpr double kAccUnit = 4.184e-4;
constexpr double kRgas = 1.987204259e-3;

// Mixed-precision payload: coordinates relative to the cell centre as int32 fixed
// point in units of 2^-25 A, so differences (and cell shifts) are exact integers and
// are rounded once when converted to FP32.  Range: |value| < 64 A.
constexpr int kFixBits = 25;
constexpr double kFix = 33554432.0;               // 2^25
constexpr float kInvFixF = 2.98023223876953125e-8f;   // 2^-25
constexpr float kInvFix2F = 8.8817841970012523e-16f;  // 2^-50

// tag of a sorted atom: global index << 4 | type << 3 | (cell x-index & 7)
__host__ __device__ inline int32_t tag_index(int32_t tag) { return tag >> 4; }
__host__ __device__ inline int32_t tag_type(int32_t tag) { return (tag >> 3) & 1; }
__host__ __device__ inline int32_t tag_cx(int32_t tag) { return tag & 7; }
constexpr int64_t kMaxAtoms = (int64_t)1 << 25;   // the LJ candidate list packs sorted index << 7

struct BoxDev {
  double L[3], invL[3];   // edges and 1/L (computed on the host)
  double cinv[3];         // M/L: cell index scale
  double edge[3];         // L/M
  int32_t M[3];
  int32_t edge_q[3];      // cell edge in fixed-point units (rint(edge * 2^25))
  double inv_mx, inv_mxy; // 1 / M[0] and 1 / (M[0] M[1]) (cell_coords)
  int32_t atom_off, n_atoms;
  int32_t cell_off, n_cells;
  int32_t blk_off;        // first per-atom block (kAtomBlock) of this box
  int32_t lj_blk_off;     // first LJ work block of this box
  int32_t cell_blk_off;   // first neighbour-list build block (kTileWaves cells) of this box
  double T0;              // <= 0: no thermostat
  double dof;             // 3N - 3
  double inv_mass;        // 1 / total mass of the box
  int64_t nl_off;         // first entry of this box's neighbour lists
  // first-level chunks of the per-box reduction (kReduceChunk block partials each)
  int32_t bd_chunk_off, bd_chunks;   // of the bonded/kinetic partials
  int32_t lj_chunk_off, lj_chunks;   // of the LJ partials (numbered after all bonded chunks)
};

// Force-field constants in the form the kernels use (built on the host).
struct FFDev {
  double mass[2];         // g/mol
  double acc_over_m[2];   // kAccUnit / mass
  double half_m_over_acc[2];  // m / (2 kAccUnit): kinetic energy factor
  // LJ per type pair t = ti * 2 + tj:
  //   force scalar  ff = r^-2 r^-6 (f12 r^-6 - f6)   (F_i = ff * (x_i - x_j))
  //   energy        E  = r^-6 (e12 r^-6 - e6)
  double f12[4], f6[4], e12[4], e6[4], ecut[4];
  double rc2;
  double kb, b0, ka, theta0, kphi, cos_phis, sin_phis;
  int32_t n_dih, excl, chain_len, uniform_lj;
  // i / chain_len = umulhi(i, chain_magic) >> chain_shift for 0 <= i < 2^25 (chain_len >= 4):
  // chain_magic = floor(2^(31 + s) / chain_len) + 1, chain_shift = s - 1, s = ceil(log2 chain_len)
  uint32_t chain_magic;
  int32_t chain_shift;
};

// First atom of atom i's chain, i - i % chain_len, without an integer division.
__device__ inline int32_t chain_first(int32_t i, const FFDev& ff) {
  return (int32_t)(__umulhi((uint32_t)i, ff.chain_magic) >> ff.chain_shift) * ff.chain_len;
}

// Cell coordinates (lc % M0, lc / M0 % M1, lc / (M0 M1)) of cell lc of box B, without
// integer division: (lc + 1/2) / M lies at least 1/(2M) from an integer, and the FP64
// product with the rounded reciprocal errs by about 2^-51 times the quotient, which is
// below that margin while the box has fewer than 2^50 cells.
struct Cell3 {
  int x, y, z;
};
__device__ inline Cell3 cell_coords(int lc, const BoxDev& B) {
  const double a = (double)lc + 0.5;
  const int qy = (int)(a * B.inv_mx);    // lc / M0
  const int qz = (int)(a * B.inv_mxy);   // lc / (M0 M1)
  return Cell3{lc - qy * B.M[0], qy - qz * B.M[1], qz};
}

// Offsets (ox, oy, oz) in [-R, R] of stencil code = (ox + R) + W ((oy + R) + W (oz + R)),
// W = 2R + 1, for 0 <= code < W^3 and W <= 15: the quotients by W and W^2 come from FP32
// products with v_rcp_f32 reciprocals (1 ulp); (code + 1/2) / W^k lies at least 1/(2 W^2)
// from an integer, far above the products' error (< 1e-4).
__device__ inline Cell3 stencil_offset(int code, int R) {
  const int W = 2 * R + 1;
  const float a = (float)code + 0.5f;
  const int q1 = (int)(a * __builtin_amdgcn_rcpf((float)W));
  const int q2 = (int)(a * __builtin_amdgcn_rcpf((float)(W * W)));
  return Cell3{code - q1 * W - R, q1 - q2 * W - R, q2 - R};
}

// double-double accumulator (sum and the rounding error carried alongside)
struct dd {
  double hi, lo;
};

__device__ inline dd dd_add(dd a, dd b) {
  double s = a.hi + b.hi;
  double bb = s - a.hi;
  double err = (a.hi - (s - bb)) + (b.hi - bb);
  return dd{s, err + (a.lo + b.lo)};
}
__device__ inline dd dd_from(double v) { return dd{v, 0.0}; }

// The views every launcher needs.
struct Views {
  int64_t N, C;            // atoms, cells (all boxes)
  int32_t n_boxes, R;
  int32_t n_atom_blocks, n_lj_blocks;
  const BoxDev* boxes;
  const int32_t* blk_box;      // [n_atom_blocks] box of each per-atom block
  const int32_t* lj_blk_box;   // [n_lj_blocks] box of each LJ work block
  double* pos;
  double* vel;
  const uint8_t* type;
  int32_t* cell;       // [N] global cell of each atom
  int32_t* slot;       // [N] arrival order within the cell (atomic)
  int32_t* cnt;        // [C]
  int32_t* cell_start; // [C + 1]
  int32_t* tmp;        // [N] unordered cell lists
  int32_t* cell_atoms; // [N] ordered cell lists
  int32_t* scell;      // [N] cell of each sorted slot
  void* payload;       // [N] int4 fixed point (mixed) / double4 (fp64): cell-centre-relative xyz + tag
  void* f_lj;          // [3N] LJ force, prec
  void* f_tot;         // [3N] total force, prec
  unsigned long long* f_acc;   // [3N] half-shell LJ force, int64 fixed point (2^-32 kcal/mol/A); zero between uses
  int32_t* scan_tiles; // [n_tiles]
  dd* part_lj;         // [n_lj_blocks * 3]: E_lj, E_lj_shifted, W_lj
  dd* part_bd;         // [kBdParts][n_atom_blocks]: E_b, E_a, E_d, W_b, KE, momentum xyz
  double* thermo;      // [n_boxes * kThermo] integrator state per box (ThermoSlot)
  double* energy;      // [n_boxes * kEnergySlots] per-box results
  int32_t* err;        // sticky error word
  // neighbour-list mode (nl_cap = 0 otherwise)
  int32_t nl_cap;              // list entries per atom (per-atom lists) or per cell (per-cell lists)
  int32_t n_cell_blocks;       // list build blocks (kTileWaves home cells each)
  const int32_t* cell_blk_box; // [n_cell_blocks] box of each build block
  uint32_t* nl_list;     // entries (sorted index << 7 | stencil code).  Per-atom lists: per
                         // box, per 64 atoms of sorted order, [nl_cap][64]: entry t of atom s
                         // at nl_off + (s/64) * 64 * nl_cap + t * 64 + s % 64 (s box-local).
                         // Per-cell lists: entry t of box-local cell c at nl_off + c * nl_cap + t
  int32_t* nl_count;     // list length per sorted slot [N] (per-atom lists) or per cell [C]
  double* x_build;       // [3N] wrapped positions at the last build (global order)
  int32_t* slot_of;      // [N] sorted slot of each atom at the last build
  void* pay_cur;         // [N] the current payload: the build's after a rebuild, refreshed every step
  int32_t* nl_flag;      // rebuild flag of the current step (raised by the update, cleared by the reduction)
  unsigned long long* nl_builds;   // list builds since init
  double nl_rl2;         // (rc + skin)^2
  double nl_half_skin2;  // (skin / 2)^2
  uint32_t* obs_part;    // [kObsBlocks * kMaxObsBins] block partials of the observables
  // two-level per-box reduction (boxes with more than kReduceChunk block partials)
  int32_t n_bd_chunks, n_lj_chunks;
  int32_t l1_bd, l1_lj;  // 1: some box has more bonded / LJ partials than one chunk
  const int2* chunk_rng; // [n_bd_chunks + n_lj_chunks] first and end partial of each chunk
  dd* part_l1;           // [n_bd_chunks + n_lj_chunks][kBdParts] chunk sums
  const void* shift_tab;  // [n_boxes][kShiftSlots] stencil shifts in payload units (int32 x3 mixed, double x3
                          // FP64): slot code = the offset of stencil code, slot kSentinelCode the sentinel's
  double* ree0;          // [n_chains * 3] end-to-end vectors at the autocorrelation's reference time
  double* ree_part;      // [n_chains * 2] per-chain terms of the autocorrelation
};

enum ErrBits : int32_t { kErrNonFinite = 1 };

constexpr int kBdParts = 8;      // block partials of the bonded kernel
constexpr int kReduceChunk = 2048;   // block partials one first-level reduction block sums
constexpr int kMaxObsBins = 2048;  // histogram bins of one observable (md.h: MD_OBS_MAX_BINS)
constexpr int kObsBlocks = 512;    // work-groups of an observable kernel (grid-stride)
constexpr int kEnergySlots = 10; // per box: E_lj, E_lj_shifted, E_b, E_a, E_d, KE, T, W, xi, E_thermostat

// Integrator state per box.  The velocity update of the next step is
//   v <- post * (pre * (v - u) + k dt a)
// with k = 1/2 (velocity Verlet: pre = the pending Berendsen factor, post = 1) or k = 1
// (leap-frog: pre = 1 - dt xi / 2, post = 1 / (1 + dt xi / 2)); u is the centre-of-mass
// velocity still to be removed (0 unless removal is on).
enum ThermoSlot { kThPre = 0, kThXi = 1, kThEta = 2, kThPost = 3, kThU = 4, kThermo = 8 };
enum Integrator { kVerletBerendsen = 0, kLeapfrogNoseHoover = 1 };

// What the bonded kernel does with the velocities: nothing (forces only), the second
// velocity-Verlet half kick, or (leap-frog) read them for the kinetic energy.
enum BondedMode { kBondedForces = 0, kBondedVerletKick = 1, kBondedLeapfrog = 2 };

// Step options the per-atom kernels need.
struct StepOpts {
  double dt;          // fs
  double tau;         // Berendsen coupling time or Nose-Hoover period, fs
  int integrator;     // Integrator
  int remove_com;     // 1: remove each box's centre-of-mass velocity every step
};

// ---- launchers (md_kernels.hip) ----
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
// gate (neighbour-list mode): a device flag; when it is non-null and reads 0 the kernel does nothing
void launch_bin_count(const Views& v, bool kick, const StepOpts& o, const FFDev& ff, bool fp32_force,
                      hipStream_t s, const int32_t* gate = nullptr);
void launch_scan(const Views& v, hipStream_t s, const int32_t* gate = nullptr);
void launch_scatter(const Views& v, hipStream_t s, const int32_t* gate = nullptr);
void launch_rank_payload(const Views& v, bool fp32, hipStream_t s, const int32_t* gate = nullptr);
void launch_bonded(const Views& v, const FFDev& ff, bool fp32, BondedMode mode, bool energy, bool com,
                   double dt, hipStream_t s);
// update: advance the integrator state (thermostat, pending COM velocity) from the sums
void launch_reduce(const Views& v, bool energy, bool update, const StepOpts& o, hipStream_t s);
// applies what is pending (Berendsen factor, COM velocity) to the velocities
void launch_finalize(const Views& v, const StepOpts& o, hipStream_t s);
// neighbour-list mode: update + displacement check (raises nl_flag past half the skin, or always
// with force_build) + payload refresh
void launch_nl_integrate(const Views& v, const StepOpts& o, const FFDev& ff, bool fp32_force, bool force_build,
                         hipStream_t s);

// ---- launchers (md_obs.hip): Section 5 observables of box b ----
void launch_obs_pairs(const Views& v, int b, int64_t n_atoms, int chain_len, int excl, double dr, int n_bins,
                      unsigned long long* out, hipStream_t s);
void launch_obs_dihedrals(const Views& v, int b, int64_t n_atoms, int chain_len, int n_bins,
                          unsigned long long* out, hipStream_t s);
void launch_obs_chains(const Views& v, const FFDev& ff, int b, int64_t n_chains, int chain_len, double* out,
                       hipStream_t s);
// end-to-end autocorrelation of box b: reference = store the current vectors as time zero;
// otherwise out[b] = sum_c R_c . R_c(0) / sum_c |R_c(0)|^2 (device)
void launch_ree(const Views& v, int b, int64_t n_chains, int chain_len, bool reference, double* out, hipStream_t s);

constexpr int kTileHomesMixed = 8;   // home atoms per pass of a mixed cell-tile wave

// ---- launchers (md_lj.hip) ----
// homes: home atoms per pass of a cell-tile wave (4, 8 or 16; mixed precision)
void launch_lj(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, int homes, hipStream_t s);
int64_t lj_blocks_for_box(int kernel, int64_t n_atoms, int64_t n_cells);
// neighbour-list mode: the list build (from the bins) and the LJ force from the list;
// the force reads the current payload (pay_cur); gate: as for the bin kernels
// kernel: MD_LJ_NLIST (per-atom lists) or MD_LJ_NLIST_TILE (per-cell lists)
void launch_nl_build(const Views& v, const FFDev& ff, bool fp32, int kernel, hipStream_t s,
                     const int32_t* gate = nullptr);
void launch_lj_nl(const Views& v, const FFDev& ff, bool fp32, int kernel, bool energy, int homes, hipStream_t s);
constexpr int kLjNlBlock = 256;   // threads per block of the list force kernel (box-aligned)
constexpr int kTileWaves = 1;     // home cells (wavefronts) per block of the cell-tile kernels
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X (one L2 each)
constexpr int kTileMaxR = 2;      // stencil radii the cell-tile kernel supports
// Stencil shift table (R <= 2: at most 125 codes).  The last slot shifts a candidate by R + 1
// cell edges in x and in y: the candidate list is padded to whole 64-lane steps with entries
// sorted index 0 | kSentinelCode, which then lie at least sqrt(2) R edges >= sqrt(2) rc from
// every home atom, so they never count and need no bounds test.
constexpr int kShiftSlots = 128;
constexpr int kSentinelCode = kShiftSlots - 1;
constexpr uint32_t kSentinelEntry = (uint32_t)kSentinelCode;

}  // namespace mdk
