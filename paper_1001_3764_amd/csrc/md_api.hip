// C ABI of the gfx950 MD library: validation, workspace layout, step sequencing,
// hipGraph capture and the autotuner.  Declarations and contracts: include/md.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "md.h"
#include "md_internal.h"

using namespace mdk;

struct md_ctx {
  md_forcefield ff{};
  int32_t n_boxes = 0, chain_len = 0;
  std::vector<int32_t> n_chains;
  std::vector<double> box, T0;
  double dt = 1.0, tau = 100.0;
  int prec = MD_PREC_MIXED;
  int R = 1, lj_kernel = MD_LJ_ATOM, use_graph = 0;
  int homes = 8;             // home atoms per pass of a cell-tile wave (mixed precision)
  int64_t N = 0;
  FFDev ffd{};
  Views v{};
  std::vector<BoxDev> hboxes;
  double* pos = nullptr;
  double* vel = nullptr;
  const uint8_t* type = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  // graphs: [energy] for the cell path; [2 * build + energy] in neighbour-list mode
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
  int integrator = MD_INT_VERLET_BERENDSEN;
  int remove_com = 0;
  std::vector<double> box_mass;   // total mass of each box (from the types at init)
  double nl_skin = 0.0;      // > 0: neighbour-list mode
  int nl_every = 1;
  int since_build = 0;       // steps since the last forced list build (nl_every > 0)
  int64_t step = 0;
  bool failed = false;
  std::string last_error;
  // allocation-free contexts (md_init_system_static): the device whose scratch array is the
  // workspace, and the take-over count of that array when this context took it (-1: caller
  // workspace)
  int scratch_dev = -1;
  uint64_t scratch_gen = 0;
};

namespace {

constexpr size_t kAlign = 256;

// Workspace of the allocation-free set-up (md_init_system_static): one array per GPU in the
// code object, MD_STATIC_WORKSPACE_BYTES, held until the process ends.  In host code its name
// is a host-side stand-in, never a device address: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device (scratch_ptr).
constexpr size_t kScratchBytes = MD_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};       // device address of scratch, per device
uint64_t g_scratch_gen[kMaxDevices] = {};    // allocation-free contexts created, per device

// An allocation-free context whose device scratch array a later md_init_system_static on the
// same device has taken over: its workspace now holds the other context's data.
bool taken_over(const md_ctx* c) {
  if (c->scratch_dev < 0) return false;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_gen[c->scratch_dev] != c->scratch_gen;
}

// A context can run while it has not failed and still owns its workspace.
bool usable(const md_ctx* c) { return !c->failed && !taken_over(c); }

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

md_status fail(md_ctx* c, md_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

md_status hip_check(md_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return MD_OK;
  return fail(c, MD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

md_status validate(const md_forcefield* ff, const md_config* cfg, std::string* why) {
  if (!ff || !cfg) { *why = "null forcefield or config"; return MD_ERR_ARG; }
  for (int t = 0; t < 2; ++t)
    if (!finite_pos(ff->mass[t]) || !finite_pos(ff->sigma[t]) || !(ff->epsilon[t] >= 0) ||
        !std::isfinite(ff->epsilon[t])) {
      *why = "mass/sigma must be > 0 and epsilon >= 0";
      return MD_ERR_ARG;
    }
  if (!std::isfinite(ff->kb) || !std::isfinite(ff->ka) || !std::isfinite(ff->kphi) ||
      !std::isfinite(ff->b0) || !std::isfinite(ff->theta0_deg) || !std::isfinite(ff->phis_deg) ||
      !finite_pos(ff->rc) || ff->n_dih < 1 || ff->n_dih > 12 || ff->excl_depth < 0) {
    *why = "bad bonded parameters, cutoff, periodicity or exclusion depth";
    return MD_ERR_ARG;
  }
  if (cfg->n_boxes < 1 || cfg->chain_len < 4 || !cfg->n_chains || !cfg->box || !cfg->T0) {
    *why = "n_boxes >= 1, chain_len >= 4 and the host arrays are required";
    return MD_ERR_ARG;
  }
  if (ff->excl_depth >= cfg->chain_len) { *why = "excl_depth must be below chain_len"; return MD_ERR_ARG; }
  if (!finite_pos(cfg->dt_fs) || !finite_pos(cfg->tau_fs)) { *why = "dt and tau must be > 0"; return MD_ERR_ARG; }
  if (cfg->precision != MD_PREC_FP64 && cfg->precision != MD_PREC_MIXED) { *why = "bad precision"; return MD_ERR_ARG; }
  if (cfg->cell_div < 0 || cfg->cell_div > 3) { *why = "cell_div must be 0..3"; return MD_ERR_ARG; }
  if (cfg->nl_skin > 0.0 ? !(cfg->lj_kernel == 0 || cfg->lj_kernel == MD_LJ_NLIST || cfg->lj_kernel == MD_LJ_NLIST_TILE)
                         : !((cfg->lj_kernel >= 0 && cfg->lj_kernel <= 3) || cfg->lj_kernel == MD_LJ_HALFSHELL)) {
    *why = "lj_kernel must be 0..3 or MD_LJ_HALFSHELL (cell path), or 0, MD_LJ_NLIST, MD_LJ_NLIST_TILE (neighbour lists)";
    return MD_ERR_ARG;
  }
  if (cfg->integrator != MD_INT_VERLET_BERENDSEN && cfg->integrator != MD_INT_LEAPFROG_NH) {
    *why = "integrator must be MD_INT_VERLET_BERENDSEN or MD_INT_LEAPFROG_NH";
    return MD_ERR_ARG;
  }
  if (cfg->remove_com != 0 && cfg->remove_com != 1) { *why = "remove_com must be 0 or 1"; return MD_ERR_ARG; }
  if (cfg->tile_homes != 0 && cfg->tile_homes != 4 && cfg->tile_homes != 8 && cfg->tile_homes != 16) {
    *why = "tile_homes must be 0, 4, 8 or 16";
    return MD_ERR_ARG;
  }
  if (!(cfg->nl_skin >= 0.0) || !std::isfinite(cfg->nl_skin)) { *why = "nl_skin must be >= 0"; return MD_ERR_ARG; }
  if (cfg->nl_skin > 0.0 && cfg->nl_every < 0) { *why = "nl_every must be >= 0"; return MD_ERR_ARG; }
  if (cfg->nl_skin > 0.0 && cfg->cell_div > kTileMaxR) { *why = "neighbour lists need cell_div <= 2"; return MD_ERR_ARG; }
  int64_t N = 0;
  for (int b = 0; b < cfg->n_boxes; ++b) {
    if (cfg->n_chains[b] < 1) { *why = "every box needs at least one chain"; return MD_ERR_ARG; }
    for (int d = 0; d < 3; ++d)
      if (!finite_pos(cfg->box[3 * b + d])) { *why = "box edges must be > 0"; return MD_ERR_ARG; }
    if (!std::isfinite(cfg->T0[b])) { *why = "T0 must be finite"; return MD_ERR_ARG; }
    N += (int64_t)cfg->n_chains[b] * cfg->chain_len;
  }
  if (N < 2 || N > kMaxAtoms) { *why = "total atoms must be in [2, 2^25]"; return MD_ERR_ARG; }
  return MD_OK;
}

int cells_per_dim(double L, int R, double rc) { return (int)std::floor(L * R / rc); }

// Distance the cell stencil must cover: the cutoff, or in neighbour-list mode the list
// radius rc + skin (cells of edge >= (rc + skin) / R).
double cell_reach(const md_forcefield* ff, const md_config* cfg) {
  return ff->rc + (cfg->nl_skin > 0.0 ? cfg->nl_skin : 0.0);
}

constexpr int64_t kMaxScanTiles = (int64_t)kScanBlock * 8;   // k_scan: each tile sums the totals before it

bool grid_ok(const md_forcefield* ff, const md_config* cfg, int R) {
  int64_t cells = 0;
  for (int b = 0; b < cfg->n_boxes; ++b) {
    int64_t nc = 1;
    for (int d = 0; d < 3; ++d) {
      const int M = cells_per_dim(cfg->box[3 * b + d], R, cell_reach(ff, cfg));
      if (M < 2 * R + 1) return false;
      nc *= M;
    }
    cells += nc;
  }
  return cells <= kMaxScanTiles * kScanTile && cells < ((int64_t)1 << 31);
}

// Mixed precision stores coordinates relative to their cell centre as int32 fixed point in
// units of 2^-25 A, and the LJ kernels take differences of such values shifted by up to R cell
// edges, or R + 1 for the padding sentinel: |x_i - x_j| in those units is at most
// (R + 2) edge + skin (the list payload drifts by up to half the skin on each side), which must
// stay below 2^31 (64 A; kept to 63 A).
bool payload_ok(const md_forcefield* ff, const md_config* cfg, int R) {
  if (cfg->precision != MD_PREC_MIXED) return true;
  const double skin = cfg->nl_skin > 0.0 ? cfg->nl_skin : 0.0;
  for (int b = 0; b < cfg->n_boxes; ++b)
    for (int d = 0; d < 3; ++d) {
      const double L = cfg->box[3 * b + d];
      const int M = cells_per_dim(L, R, cell_reach(ff, cfg));
      if (M < 1 || (R + 2) * (L / M) + skin >= 63.0) return false;
    }
  return true;
}

struct Plan {
  int64_t N = 0, C = 0;
  int32_t n_boxes = 0, n_atom_blocks = 0, n_lj_blocks = 0, n_tiles = 0;
  int32_t n_cell_blocks = 0, nl_cap = 0;   // neighbour-list mode
  int32_t n_bd_chunks = 0, n_lj_chunks = 0, l1_bd = 0, l1_lj = 0;   // two-level reduction
  std::vector<int32_t> chunk_rng;           // [2 * chunks] first and end partial
  int64_t nl_entries = 0;
  bool half = false;                        // half-shell LJ: fixed-point force accumulators
  int prec = 0;
  int chain_len = 1;
  std::vector<BoxDev> boxes;
};

// List capacity (a list that fills up is reported as MD_ERR_NLIST).  Per-atom lists: the
// pairs within rc + skin at the densest box's density, 1.5x plus 64.  Per-cell lists: the
// atoms that can lie within rc + skin of a cell, i.e. in the cell grown by rc + skin (a box
// with rounded edges: V = e0 e1 e2 + 2 r (e0 e1 + e1 e2 + e2 e0) + pi r^2 (e0 + e1 + e2)
// + 4/3 pi r^3), at the box's density, 1.25x plus 64, the largest over the boxes.
int32_t nl_capacity(const md_forcefield* ff, const md_config* cfg, int R, int kernel) {
  const double rl = ff->rc + cfg->nl_skin;
  double need = 0.0;
  for (int b = 0; b < cfg->n_boxes; ++b) {
    const double* L = cfg->box + 3 * b;
    const double rho = (double)cfg->n_chains[b] * cfg->chain_len / (L[0] * L[1] * L[2]);
    if (kernel == MD_LJ_NLIST_TILE) {
      double e[3];
      for (int d = 0; d < 3; ++d) e[d] = L[d] / cells_per_dim(L[d], R, cell_reach(ff, cfg));
      const double V = e[0] * e[1] * e[2] + 2.0 * rl * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0]) +
                       M_PI * rl * rl * (e[0] + e[1] + e[2]) + 4.0 / 3.0 * M_PI * rl * rl * rl;
      need = std::max(need, 1.25 * V * rho + 64.0);
    } else {
      need = std::max(need, 1.5 * 4.0 / 3.0 * M_PI * rl * rl * rl * rho + 64.0);
    }
  }
  const int q = kernel == MD_LJ_NLIST_TILE ? 64 : 16;
  return (int32_t)((need + q - 1) / q) * q;
}

Plan make_plan(const md_forcefield* ff, const md_config* cfg, int R, int kernel) {
  Plan p;
  p.n_boxes = cfg->n_boxes;
  p.prec = cfg->precision;
  p.chain_len = cfg->chain_len;
  const bool nl = cfg->nl_skin > 0.0;
  p.half = !nl && kernel == MD_LJ_HALFSHELL;
  if (nl) {
    if (kernel != MD_LJ_NLIST_TILE) kernel = MD_LJ_NLIST;
    p.nl_cap = nl_capacity(ff, cfg, R, kernel);
  }
  int64_t atom = 0, cell = 0, blk = 0, lblk = 0, cblk = 0, nle = 0;
  for (int b = 0; b < cfg->n_boxes; ++b) {
    BoxDev B{};
    const int64_t n = (int64_t)cfg->n_chains[b] * cfg->chain_len;
    int64_t nc = 1;
    for (int d = 0; d < 3; ++d) {
      const double L = cfg->box[3 * b + d];
      const int M = cells_per_dim(L, R, cell_reach(ff, cfg));
      B.L[d] = L;
      B.invL[d] = 1.0 / L;
      B.M[d] = M;
      B.cinv[d] = (double)M / L;
      B.edge[d] = L / (double)M;
      B.edge_q[d] = (int32_t)std::lrint(B.edge[d] * kFix);
      nc *= M;
    }
    B.inv_mx = 1.0 / (double)B.M[0];
    B.inv_mxy = 1.0 / ((double)B.M[0] * (double)B.M[1]);
    B.atom_off = (int32_t)atom;
    B.n_atoms = (int32_t)n;
    B.cell_off = (int32_t)cell;
    B.n_cells = (int32_t)nc;
    B.blk_off = (int32_t)blk;
    B.lj_blk_off = (int32_t)lblk;
    B.cell_blk_off = (int32_t)cblk;
    B.nl_off = nle;
    B.T0 = cfg->T0[b];
    B.dof = (double)(3 * n - 3);
    atom += n;
    cell += nc;
    blk += (n + kAtomBlock - 1) / kAtomBlock;
    lblk += lj_blocks_for_box(kernel, n, nc);
    if (nl) {
      cblk += (nc + kTileWaves - 1) / kTileWaves;
      nle += (kernel == MD_LJ_NLIST_TILE ? nc : (n + 63) / 64 * 64) * (int64_t)p.nl_cap;
    }
    p.boxes.push_back(B);
  }
  p.n_cell_blocks = (int32_t)cblk;
  p.nl_entries = nle;
  p.N = atom;
  p.C = cell;
  p.n_atom_blocks = (int32_t)blk;
  p.n_lj_blocks = (int32_t)lblk;
  p.n_tiles = (int32_t)((cell + kScanTile - 1) / kScanTile);
  // first-level chunks of the per-box reduction: bonded partials of every box, then LJ partials
  for (int pass = 0; pass < 2; ++pass)
    for (int b = 0; b < p.n_boxes; ++b) {
      BoxDev& B = p.boxes[b];
      const int32_t first = pass == 0 ? B.blk_off : B.lj_blk_off;
      const int32_t end = pass == 0 ? (b + 1 < p.n_boxes ? p.boxes[b + 1].blk_off : p.n_atom_blocks)
                                    : (b + 1 < p.n_boxes ? p.boxes[b + 1].lj_blk_off : p.n_lj_blocks);
      const int32_t n = (end - first + kReduceChunk - 1) / kReduceChunk;
      (pass == 0 ? B.bd_chunk_off : B.lj_chunk_off) = (int32_t)(p.chunk_rng.size() / 2);
      (pass == 0 ? B.bd_chunks : B.lj_chunks) = n;
      for (int32_t k = 0; k < n; ++k) {
        p.chunk_rng.push_back(first + k * kReduceChunk);
        p.chunk_rng.push_back(std::min(end, first + (k + 1) * kReduceChunk));
      }
      if (n > 1) (pass == 0 ? p.l1_bd : p.l1_lj) = 1;
      (pass == 0 ? p.n_bd_chunks : p.n_lj_chunks) += n;
    }
  return p;
}

// Carves the workspace (base may be null to only measure).
size_t carve(const Plan& p, char* base, Views* v) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* r = base ? base + off : nullptr;
    off += align_up(bytes > 0 ? bytes : 1);
    return r;
  };
  const size_t fsz = p.prec == MD_PREC_MIXED ? 4 : 8;
  const size_t psz = p.prec == MD_PREC_MIXED ? 16 : 32;
  Views t{};
  t.N = p.N;
  t.C = p.C;
  t.n_boxes = p.n_boxes;
  t.n_atom_blocks = p.n_atom_blocks;
  t.n_lj_blocks = p.n_lj_blocks;
  t.boxes = (const BoxDev*)take(sizeof(BoxDev) * p.n_boxes);
  t.blk_box = (const int32_t*)take(4 * (size_t)p.n_atom_blocks);
  t.lj_blk_box = (const int32_t*)take(4 * (size_t)p.n_lj_blocks);
  t.cell = (int32_t*)take(4 * (size_t)p.N);
  t.slot = (int32_t*)take(4 * (size_t)p.N);
  t.cnt = (int32_t*)take(4 * (size_t)p.C);
  t.cell_start = (int32_t*)take(4 * (size_t)(p.C + 1));
  t.tmp = (int32_t*)take(4 * (size_t)p.N);
  t.cell_atoms = (int32_t*)take(4 * (size_t)p.N);
  t.scell = (int32_t*)take(4 * (size_t)p.N);
  t.payload = take(psz * (size_t)p.N);
  t.f_lj = take(3 * fsz * (size_t)p.N);
  t.f_tot = take(3 * fsz * (size_t)p.N);
  if (p.half) t.f_acc = (unsigned long long*)take(24 * (size_t)p.N);
  t.scan_tiles = (int32_t*)take(4 * (size_t)p.n_tiles);
  t.part_lj = (dd*)take(sizeof(dd) * 3 * (size_t)p.n_lj_blocks);
  t.part_bd = (dd*)take(sizeof(dd) * kBdParts * (size_t)p.n_atom_blocks);
  t.thermo = (double*)take(8 * kThermo * (size_t)p.n_boxes);
  t.energy = (double*)take(8 * kEnergySlots * (size_t)p.n_boxes);
  t.err = (int32_t*)take(4);
  t.obs_part = (uint32_t*)take(4 * (size_t)kObsBlocks * kMaxObsBins);
  t.shift_tab = take((p.prec == MD_PREC_MIXED ? 12 : 24) * (size_t)kShiftSlots * p.n_boxes);
  t.n_bd_chunks = p.n_bd_chunks;
  t.n_lj_chunks = p.n_lj_chunks;
  t.l1_bd = p.l1_bd;
  t.l1_lj = p.l1_lj;
  t.chunk_rng = (const int2*)take(4 * p.chunk_rng.size());
  t.part_l1 = (dd*)take(sizeof(dd) * kBdParts * (size_t)(p.n_bd_chunks + p.n_lj_chunks));
  t.ree0 = (double*)take(24 * (size_t)(p.N / p.chain_len));
  t.ree_part = (double*)take(16 * (size_t)(p.N / p.chain_len));
  if (p.nl_cap) {
    t.nl_cap = p.nl_cap;
    t.n_cell_blocks = p.n_cell_blocks;
    t.cell_blk_box = (const int32_t*)take(4 * (size_t)p.n_cell_blocks);
    t.nl_list = (uint32_t*)take(4 * (size_t)p.nl_entries);
    t.nl_count = (int32_t*)take(4 * (size_t)std::max(p.N, p.C));
    t.x_build = (double*)take(24 * (size_t)p.N);
    t.slot_of = (int32_t*)take(4 * (size_t)p.N);
    t.pay_cur = take(psz * (size_t)p.N);
    t.nl_flag = (int32_t*)take(4);
    t.nl_builds = (unsigned long long*)take(8);
  }
  if (v) *v = t;
  return off;
}

FFDev make_ffdev(const md_forcefield* ff, int chain_len) {
  FFDev d{};
  for (int t = 0; t < 2; ++t) {
    d.mass[t] = ff->mass[t];
    d.acc_over_m[t] = kAccUnit / ff->mass[t];
    d.half_m_over_acc[t] = 0.5 * ff->mass[t] / kAccUnit;
  }
  d.uniform_lj = 1;
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj) {
      const int t = ti * 2 + tj;
      const double sig = 0.5 * (ff->sigma[ti] + ff->sigma[tj]);   // Lorentz-Berthelot
      const double eps = std::sqrt(ff->epsilon[ti] * ff->epsilon[tj]);
      const double s6 = sig * sig * sig * sig * sig * sig;
      const double ljp1 = 4.0 * eps * s6;          // 4 eps sigma^6
      const double ljp2 = 4.0 * eps * s6 * s6;     // 4 eps sigma^12
      d.e12[t] = ljp2;
      d.e6[t] = ljp1;
      d.f12[t] = 12.0 * ljp2;
      d.f6[t] = 6.0 * ljp1;
      const double rc6 = std::pow(ff->rc, 6.0);
      d.ecut[t] = ljp2 / (rc6 * rc6) - ljp1 / rc6;
    }
  for (int t = 1; t < 4; ++t)
    if (d.f12[t] != d.f12[0] || d.f6[t] != d.f6[0]) d.uniform_lj = 0;
  d.rc2 = ff->rc * ff->rc;
  d.kb = ff->kb;
  d.b0 = ff->b0;
  d.ka = ff->ka;
  d.theta0 = ff->theta0_deg * M_PI / 180.0;
  d.kphi = ff->kphi;
  d.cos_phis = std::cos(ff->phis_deg * M_PI / 180.0);
  d.sin_phis = std::sin(ff->phis_deg * M_PI / 180.0);
  d.n_dih = ff->n_dih;
  d.excl = ff->excl_depth;
  d.chain_len = chain_len;
  int s = 0;
  while ((1LL << s) < chain_len) ++s;
  d.chain_magic = (uint32_t)(((uint64_t)1 << (31 + s)) / (uint64_t)chain_len + 1);
  d.chain_shift = s - 1;
  return d;
}

md_status check_launch(md_ctx* c, const char* what) { return hip_check(c, hipGetLastError(), what); }

// The end-to-end vectors of every chain: stored as the reference (reference), or correlated
// with it into out[n_boxes] (device).
void enqueue_ree(md_ctx* c, bool reference, double* out) {
  for (int b = 0; b < c->n_boxes; ++b) launch_ree(c->v, b, c->n_chains[b], c->chain_len, reference, out, c->stream);
}

StepOpts opts(const md_ctx* c) {
  StepOpts o;
  o.dt = c->dt;
  o.tau = c->tau;
  o.integrator = c->integrator;
  o.remove_com = c->remove_com;
  return o;
}

// Lays out the workspace for stencil radius R and kernel k, uploads the tables and
// clears the counters.  Does not touch positions or velocities.
md_status configure(md_ctx* c, const md_config* cfg, int R, int kernel) {
  Plan p = make_plan(&c->ff, cfg, R, kernel);
  for (int b = 0; b < p.n_boxes; ++b) p.boxes[b].inv_mass = 1.0 / c->box_mass[b];
  Views v{};
  const size_t need = carve(p, nullptr, nullptr);
  if (need > c->ws_bytes) return fail(c, MD_ERR_WORKSPACE, "workspace too small for this configuration");
  carve(p, c->ws, &v);
  v.R = R;
  v.pos = c->pos;
  v.vel = c->vel;
  v.type = c->type;
  std::vector<int32_t> bb(p.n_atom_blocks), lb(p.n_lj_blocks), cb(p.n_cell_blocks);
  for (int b = 0; b < p.n_boxes; ++b) {
    const int32_t e1 = b + 1 < p.n_boxes ? p.boxes[b + 1].blk_off : p.n_atom_blocks;
    for (int32_t k = p.boxes[b].blk_off; k < e1; ++k) bb[k] = b;
    const int32_t e2 = b + 1 < p.n_boxes ? p.boxes[b + 1].lj_blk_off : p.n_lj_blocks;
    for (int32_t k = p.boxes[b].lj_blk_off; k < e2; ++k) lb[k] = b;
    const int32_t e3 = b + 1 < p.n_boxes ? p.boxes[b + 1].cell_blk_off : p.n_cell_blocks;
    for (int32_t k = p.boxes[b].cell_blk_off; k < e3; ++k) cb[k] = b;
  }
  if (p.nl_cap) {
    const double rl = c->ff.rc + cfg->nl_skin;
    v.nl_rl2 = rl * rl;
    v.nl_half_skin2 = 0.25 * cfg->nl_skin * cfg->nl_skin;
  }
  md_status st;
  // pageable sources: hipMemcpy (synchronous) so the host vectors may go away
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return st;
  if ((st = hip_check(c, hipMemcpy((void*)v.boxes, p.boxes.data(), sizeof(BoxDev) * p.n_boxes,
                                   hipMemcpyHostToDevice), "upload boxes")))
    return st;
  if ((st = hip_check(c, hipMemcpy((void*)v.blk_box, bb.data(), 4 * bb.size(), hipMemcpyHostToDevice),
                      "upload block table")))
    return st;
  if ((st = hip_check(c, hipMemcpy((void*)v.lj_blk_box, lb.data(), 4 * lb.size(), hipMemcpyHostToDevice),
                      "upload LJ block table")))
    return st;
  if (p.nl_cap &&
      (st = hip_check(c, hipMemcpy((void*)v.cell_blk_box, cb.data(), 4 * cb.size(), hipMemcpyHostToDevice),
                      "upload list build block table")))
    return st;
  if ((st = hip_check(c, hipMemcpy((void*)v.chunk_rng, p.chunk_rng.data(), 4 * p.chunk_rng.size(),
                                   hipMemcpyHostToDevice), "upload reduction chunks")))
    return st;
  if (R <= kTileMaxR) {
    // stencil shifts per box in the payload's units, and the sentinel slot
    const int W = 2 * R + 1;
    std::vector<int32_t> qi((size_t)3 * kShiftSlots * p.n_boxes, 0);
    std::vector<double> qd((size_t)3 * kShiftSlots * p.n_boxes, 0.0);
    for (int b = 0; b < p.n_boxes; ++b)
      for (int code = 0; code < kShiftSlots; ++code) {
        int o[3] = {R + 1, R + 1, 0};   // the sentinel
        if (code < W * W * W) {
          o[0] = code % W - R;
          o[1] = code / W % W - R;
          o[2] = code / (W * W) - R;
        } else if (code != kSentinelCode) {
          continue;
        }
        const size_t at = ((size_t)b * kShiftSlots + code) * 3;
        for (int d = 0; d < 3; ++d) {
          qi[at + d] = o[d] * p.boxes[b].edge_q[d];
          qd[at + d] = o[d] * p.boxes[b].edge[d];
        }
      }
    const bool mixed = p.prec == MD_PREC_MIXED;
    if ((st = hip_check(c, hipMemcpy(const_cast<void*>(v.shift_tab), mixed ? (const void*)qi.data() : (const void*)qd.data(),
                                     mixed ? 4 * qi.size() : 8 * qd.size(), hipMemcpyHostToDevice),
                        "upload stencil shifts")))
      return st;
  }
  std::vector<double> th((size_t)kThermo * p.n_boxes, 0.0);
  for (int b = 0; b < p.n_boxes; ++b) th[(size_t)b * kThermo + kThPre] = th[(size_t)b * kThermo + kThPost] = 1.0;
  if ((st = hip_check(c, hipMemcpy(v.thermo, th.data(), 8 * th.size(), hipMemcpyHostToDevice),
                      "upload integrator state")))
    return st;
  launch_fill_i32(v.cnt, p.C, 0, c->stream);
  launch_fill_i32(v.err, 1, 0, c->stream);
  if (v.f_acc) launch_fill_i32((int32_t*)v.f_acc, 6 * p.N, 0, c->stream);
  if (v.nl_flag) {
    launch_fill_i32(v.nl_flag, 1, 0, c->stream);
    launch_fill_i32((int32_t*)v.nl_builds, 2, 0, c->stream);
  }
  launch_fill_f64(v.energy, kEnergySlots * (int64_t)p.n_boxes, 0.0, c->stream);
  if ((st = check_launch(c, "clear workspace"))) return st;
  c->v = v;
  c->hboxes = p.boxes;
  c->R = R;
  c->lj_kernel = p.nl_cap && kernel != MD_LJ_NLIST_TILE ? MD_LJ_NLIST : kernel;
  c->since_build = 0;
  return MD_OK;
}

bool nl_mode(const md_ctx* c) { return c->v.nl_cap > 0; }

// Bins (and, in neighbour-list mode, the list) from the current positions.
void enqueue_rebuild(md_ctx* c, hipStream_t s, bool kick) {
  const bool fp32 = c->prec == MD_PREC_MIXED;
  launch_bin_count(c->v, kick, opts(c), c->ffd, fp32, s);
  launch_scan(c->v, s);
  launch_scatter(c->v, s);
  launch_rank_payload(c->v, fp32, s);
  if (nl_mode(c)) launch_nl_build(c->v, c->ffd, fp32, c->lj_kernel, s);
}

BondedMode bonded_mode(const md_ctx* c, bool step) {
  if (!step) return kBondedForces;
  return c->integrator == MD_INT_LEAPFROG_NH ? kBondedLeapfrog : kBondedVerletKick;
}

// kick: part of a step (the bonded kernel then kicks or reads the velocities).
void enqueue_forces(md_ctx* c, hipStream_t s, bool kick, bool energy) {
  const bool fp32 = c->prec == MD_PREC_MIXED;
  if (nl_mode(c))
    launch_lj_nl(c->v, c->ffd, fp32, c->lj_kernel, energy, c->homes, s);
  else
    launch_lj(c->v, c->ffd, fp32, c->lj_kernel, energy, c->homes, s);
  launch_bonded(c->v, c->ffd, fp32, bonded_mode(c, kick), energy, kick && c->remove_com, c->dt, s);
}

// One step.  Cell path: bins rebuilt, then forces.  Neighbour-list mode: the update raises the
// device's rebuild flag when an atom has moved more than half the skin since the last build (or
// always, force_build), and the bin and list kernels that follow do their work only when it is
// raised, so one captured sequence serves every step; the reduction clears the flag.
void enqueue_step(md_ctx* c, hipStream_t s, bool energy, bool force_build = false) {
  const bool fp32 = c->prec == MD_PREC_MIXED;
  if (nl_mode(c)) {
    const int32_t* gate = c->v.nl_flag;
    launch_nl_integrate(c->v, opts(c), c->ffd, fp32, force_build, s);
    launch_bin_count(c->v, false, opts(c), c->ffd, fp32, s, gate);
    launch_scan(c->v, s, gate);
    launch_scatter(c->v, s, gate);
    launch_rank_payload(c->v, fp32, s, gate);
    launch_nl_build(c->v, c->ffd, fp32, c->lj_kernel, s, gate);
  } else {
    enqueue_rebuild(c, s, true);
  }
  enqueue_forces(c, s, true, energy);
  launch_reduce(c->v, energy, true, opts(c), s);
}

// Neighbour-list mode with nl_every > 0: whether the next step rebuilds regardless of the
// displacements (nl_every steps after the last such build).
bool next_step_forced(const md_ctx* c) { return nl_mode(c) && c->nl_every > 0 && c->since_build + 1 >= c->nl_every; }

void advance_build_counter(md_ctx* c, bool forced) { c->since_build = forced ? 0 : c->since_build + 1; }

void destroy_graphs(md_ctx* c) {
  for (int k = 0; k < 4; ++k) {
    if (c->exec[k]) (void)hipGraphExecDestroy(c->exec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->exec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

md_status capture_graphs(md_ctx* c) {
  destroy_graphs(c);
  md_status st;
  if (!c->cap && (st = hip_check(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "capture stream")))
    return st;
  for (int k = 0; k < (nl_mode(c) ? 4 : 2); ++k) {
    if ((st = hip_check(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "begin capture")))
      return st;
    enqueue_step(c, c->cap, (k & 1) != 0, k >= 2);
    hipError_t le = hipGetLastError();
    hipError_t e = hipStreamEndCapture(c->cap, &c->graph[k]);
    if ((st = hip_check(c, le, "launch during capture"))) return st;
    if ((st = hip_check(c, e, "end capture"))) return st;
    if ((st = hip_check(c, hipGraphInstantiate(&c->exec[k], c->graph[k], nullptr, nullptr, 0),
                        "instantiate graph")))
      return st;
  }
  return MD_OK;
}

// A candidate replaces the best so far only when it is faster by this fraction: candidates
// within timing noise of each other (the cell tile with and without branching) then resolve
// to the same choice on every run.
constexpr float kTuneMargin = 0.03f;

// Times rebuild + forces for each candidate and keeps the fastest (see kTuneMargin).
md_status autotune(md_ctx* c, const md_config* cfg, int* bestR, int* bestK, int* bestH) {
  std::vector<int> Rs, Ks;
  if (cfg->cell_div) Rs.push_back(cfg->cell_div);
  else
    for (int R = 1; R <= 2; ++R)
      if (grid_ok(&c->ff, cfg, R) && payload_ok(&c->ff, cfg, R)) Rs.push_back(R);
  if (cfg->nl_skin > 0.0) {
    if (cfg->lj_kernel) {
      Ks.push_back(cfg->lj_kernel);
    } else {
      Ks.push_back(MD_LJ_NLIST);
      Ks.push_back(MD_LJ_NLIST_TILE);
    }
    Rs.erase(std::remove_if(Rs.begin(), Rs.end(), [](int R) { return R > kTileMaxR; }), Rs.end());
  } else if (cfg->lj_kernel) Ks.push_back(cfg->lj_kernel);
  else {
    Ks.push_back(MD_LJ_ATOM);
    Ks.push_back(MD_LJ_CELLTILE);
    if (cfg->precision == MD_PREC_MIXED) Ks.push_back(MD_LJ_CELLTILE_NB);
  }
  if (Rs.empty()) return fail(c, MD_ERR_BOX_TOO_SMALL, "no stencil fits every box");
  hipEvent_t e0, e1;
  md_status st;
  if ((st = hip_check(c, hipEventCreate(&e0), "event"))) return st;
  if ((st = hip_check(c, hipEventCreate(&e1), "event"))) return st;
  float best = 1e30f;
  *bestR = Rs[0];
  *bestK = Ks[0];
  *bestH = cfg->tile_homes ? cfg->tile_homes : 8;
  // homes per wave of the mixed cell-tile kernels (atoms-per-wavefront): tuned unless given
  const bool tile_tuned = cfg->precision == MD_PREC_MIXED && cfg->tile_homes == 0;
  std::vector<std::pair<int, int>> KH;
  for (int K : Ks) {
    const bool tile = K == MD_LJ_CELLTILE || K == MD_LJ_CELLTILE_NB || K == MD_LJ_NLIST_TILE;
    if (tile && tile_tuned)
      for (int H : {4, 8, 16}) KH.push_back({K, H});
    else
      KH.push_back({K, *bestH});
  }
  for (int R : Rs)
    for (auto kh : KH) {
      const int K = kh.first;
      if (Rs.size() * KH.size() == 1) break;
      if (K >= MD_LJ_CELLTILE && R > kTileMaxR) continue;
      c->homes = kh.second;
      if ((st = configure(c, cfg, R, K))) break;
      enqueue_rebuild(c, c->stream, false);
      enqueue_forces(c, c->stream, false, false);
      (void)hipEventRecord(e0, c->stream);
      for (int rep = 0; rep < 3; ++rep) {
        // neighbour lists: one build serves several force evaluations (all of them from the
        // build's payload: nothing has refreshed the per-step payload here)
        if (rep == 0 || !nl_mode(c)) enqueue_rebuild(c, c->stream, false);
        enqueue_forces(c, c->stream, false, false);
      }
      (void)hipEventRecord(e1, c->stream);
      if ((st = hip_check(c, hipEventSynchronize(e1), "autotune sync"))) break;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best * (1.0f - kTuneMargin)) {
        best = ms;
        *bestR = R;
        *bestK = K;
        *bestH = kh.second;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace

extern "C" {

md_status md_workspace_bytes(const md_forcefield* ff, const md_config* cfg, size_t* bytes) {
  std::string why;
  if (!bytes) return MD_ERR_ARG;
  md_status st = validate(ff, cfg, &why);
  if (st) return st;
  size_t best = 0;
  bool any = false, grid_fits = false;
  for (int R = 1; R <= 3; ++R) {
    if (cfg->cell_div && cfg->cell_div != R) continue;
    if (!cfg->cell_div && R > 2) continue;
    if (!grid_ok(ff, cfg, R)) continue;
    grid_fits = true;
    if (!payload_ok(ff, cfg, R)) continue;
    for (int K = 1; K <= MD_LJ_HALFSHELL; ++K) {
      if (cfg->lj_kernel ? cfg->lj_kernel != K : K == MD_LJ_HALFSHELL) continue;
      if ((cfg->nl_skin > 0.0) != (K == MD_LJ_NLIST || K == MD_LJ_NLIST_TILE)) continue;
      if (K >= MD_LJ_CELLTILE && R > kTileMaxR) continue;
      best = std::max(best, carve(make_plan(ff, cfg, R, K), nullptr, nullptr));
      any = true;
    }
  }
  if (!any) return grid_fits ? MD_ERR_ARG : MD_ERR_BOX_TOO_SMALL;   // ARG: the int32 payload would overflow
  *bytes = best;
  return MD_OK;
}

// md_init_system and md_init_system_static.  scratch_dev >= 0: the workspace is that device's
// scratch array (its take-over count is recorded in the context).
static md_status init_impl(const md_forcefield* ff, const md_config* cfg, double* pos, double* vel,
                           const uint8_t* type, void* workspace, size_t ws_bytes, void* stream, md_ctx** out,
                           int scratch_dev, uint64_t scratch_gen) {
  if (!out) return MD_ERR_ARG;
  *out = nullptr;
  std::string why;
  md_status st = validate(ff, cfg, &why);
  if (st) return st;
  if (!pos || !vel || !type || !workspace) return MD_ERR_ARG;
  if (((uintptr_t)workspace) % kAlign) return MD_ERR_WORKSPACE;
  if (cfg->cell_div && !grid_ok(ff, cfg, cfg->cell_div)) return MD_ERR_BOX_TOO_SMALL;
  if (!cfg->cell_div && !grid_ok(ff, cfg, 1)) return MD_ERR_BOX_TOO_SMALL;
  if (cfg->cell_div && !payload_ok(ff, cfg, cfg->cell_div)) return MD_ERR_ARG;
  if (cfg->lj_kernel >= MD_LJ_CELLTILE && cfg->cell_div > kTileMaxR) return MD_ERR_ARG;
  size_t need = 0;
  if ((st = md_workspace_bytes(ff, cfg, &need))) return st;
  if (ws_bytes < need) return MD_ERR_WORKSPACE;
  md_ctx* c = new (std::nothrow) md_ctx();
  if (!c) return MD_ERR_ARG;
  c->ff = *ff;
  c->n_boxes = cfg->n_boxes;
  c->chain_len = cfg->chain_len;
  c->n_chains.assign(cfg->n_chains, cfg->n_chains + cfg->n_boxes);
  c->box.assign(cfg->box, cfg->box + 3 * cfg->n_boxes);
  c->T0.assign(cfg->T0, cfg->T0 + cfg->n_boxes);
  c->dt = cfg->dt_fs;
  c->tau = cfg->tau_fs;
  c->prec = cfg->precision;
  c->use_graph = cfg->use_graph ? 1 : 0;
  c->integrator = cfg->integrator;
  c->remove_com = cfg->remove_com;
  c->nl_skin = cfg->nl_skin;
  c->nl_every = cfg->nl_skin > 0.0 ? cfg->nl_every : 1;
  c->pos = pos;
  c->vel = vel;
  c->type = type;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->stream = (hipStream_t)stream;
  c->scratch_dev = scratch_dev;
  c->scratch_gen = scratch_gen;
  c->ffd = make_ffdev(ff, cfg->chain_len);
  {
    // total mass per box, for the centre-of-mass velocity
    c->N = 0;
    for (int b = 0; b < cfg->n_boxes; ++b) c->N += (int64_t)cfg->n_chains[b] * cfg->chain_len;
    std::vector<uint8_t> ht((size_t)c->N);
    st = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (!st) st = hip_check(c, hipMemcpy(ht.data(), type, (size_t)c->N, hipMemcpyDeviceToHost), "read types");
    if (st) {
      std::fprintf(stderr, "md_init_system: %s\n", c->last_error.c_str());
      delete c;
      return st;
    }
    for (int64_t i = 0; i < c->N; ++i)
      if (ht[i] > 1) {   // the force field has two atom types (Table I: CH2, CH3)
        std::fprintf(stderr, "md_init_system: atom %lld has type %d (types are 0 and 1)\n", (long long)i,
                     (int)ht[i]);
        delete c;
        return MD_ERR_ARG;
      }
    int64_t a = 0;
    for (int b = 0; b < cfg->n_boxes; ++b) {
      const int64_t n = (int64_t)cfg->n_chains[b] * cfg->chain_len;
      double m = 0.0;
      for (int64_t i = 0; i < n; ++i) m += ff->mass[ht[a + i]];
      c->box_mass.push_back(m);
      a += n;
    }
  }
  md_config local = *cfg;
  local.n_chains = c->n_chains.data();
  local.box = c->box.data();
  local.T0 = c->T0.data();
  int R = cfg->cell_div ? cfg->cell_div : 1;
  int K = cfg->lj_kernel ? cfg->lj_kernel : MD_LJ_ATOM;
  int H = cfg->tile_homes ? cfg->tile_homes : 8;
  if (!cfg->cell_div || !cfg->lj_kernel) st = autotune(c, &local, &R, &K, &H);
  c->homes = H;
  if (!st) st = configure(c, &local, R, K);
  if (!st) {
    enqueue_rebuild(c, c->stream, false);
    enqueue_forces(c, c->stream, false, true);
    launch_reduce(c->v, true, false, opts(c), c->stream);
    enqueue_ree(c, true, nullptr);   // the end-to-end autocorrelation's reference: the initial state
    st = check_launch(c, "initial forces");
  }
  if (!st && c->use_graph) st = capture_graphs(c);
  if (!st) st = hip_check(c, hipStreamSynchronize(c->stream), "init sync");
  if (st) {
    std::fprintf(stderr, "md_init_system: %s\n", c->last_error.c_str());
    destroy_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return st;
  }
  *out = c;
  return MD_OK;
}

md_status md_init_system(const md_forcefield* ff, const md_config* cfg, double* pos, double* vel,
                         const uint8_t* type, void* workspace, size_t ws_bytes, void* stream,
                         md_ctx** out) {
  return init_impl(ff, cfg, pos, vel, type, workspace, ws_bytes, stream, out, -1, 0);
}

md_status md_init_system_static(const md_forcefield* ff, const md_config* cfg, double* pos, double* vel,
                                const uint8_t* type, void* stream, md_ctx** out) {
  if (!out) return MD_ERR_ARG;
  *out = nullptr;
  std::string why;
  md_status st = validate(ff, cfg, &why);
  if (st) return st;
  if (!pos || !vel || !type) return MD_ERR_ARG;
  // no graph (instantiating one allocates) and no autotuning (its timing events): both choices
  // must come from the caller
  if (cfg->use_graph || cfg->cell_div == 0 || cfg->lj_kernel == 0) return MD_ERR_ARG;
  size_t need = 0;
  if ((st = md_workspace_bytes(ff, cfg, &need))) return st;
  if (need > kScratchBytes) return MD_ERR_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MD_ERR_HIP;
  uint64_t gen = 0;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      // once per device, with that device current: the device address of this device's copy
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MD_ERR_HIP;
      g_scratch_ptr[dev] = p;
    }
    ws = g_scratch_ptr[dev];
    gen = ++g_scratch_gen[dev];   // earlier allocation-free contexts of this device stop here
  }
  return init_impl(ff, cfg, pos, vel, type, ws, kScratchBytes, stream, out, dev, gen);
}

md_status md_rebuild_bins(md_ctx* c) {
  if (!c) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  enqueue_rebuild(c, c->stream, false);
  c->since_build = 0;
  return check_launch(c, "rebuild bins");
}

md_status md_compute_forces(md_ctx* c, int32_t with_energy) {
  if (!c) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  enqueue_forces(c, c->stream, false, with_energy != 0);
  if (with_energy) launch_reduce(c->v, true, false, opts(c), c->stream);
  return check_launch(c, "compute forces");
}

md_status md_step(md_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  if (n_steps == 0) return MD_OK;
  md_status st;
  for (int32_t k = 0; k < n_steps; ++k) {
    const bool last = k == n_steps - 1;
    const bool forced = next_step_forced(c);
    if (c->use_graph) {
      const int g = (forced ? 2 : 0) + (last ? 1 : 0);
      if ((st = hip_check(c, hipGraphLaunch(c->exec[g], c->stream), "graph launch"))) return st;
    } else {
      enqueue_step(c, c->stream, last, forced);
    }
    advance_build_counter(c, forced);
  }
  launch_finalize(c->v, opts(c), c->stream);
  c->step += n_steps;
  return check_launch(c, "step");
}

md_status md_step_timed(md_ctx* c, int32_t n_steps, double* ms_out) {
  if (!c || n_steps < 0 || !ms_out) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  if (n_steps == 0) return MD_OK;
  md_status st;
  const int P = MD_N_PHASES;
  std::vector<hipEvent_t> ev((size_t)n_steps * P * 2, nullptr);
  for (auto& e : ev)
    if ((st = hip_check(c, hipEventCreate(&e), "event create"))) {
      for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
      return st;
    }
  const bool fp32 = c->prec == MD_PREC_MIXED;
  hipStream_t s = c->stream;
  for (int32_t k = 0; k < n_steps; ++k) {
    const bool last = k == n_steps - 1;
    const bool forced = next_step_forced(c);
    const bool nl = nl_mode(c);
    const int32_t* gate = nl ? c->v.nl_flag : nullptr;
    hipEvent_t* e = &ev[(size_t)k * P * 2];
    (void)hipEventRecord(e[0], s);
    if (nl) launch_nl_integrate(c->v, opts(c), c->ffd, fp32, forced, s);
    launch_bin_count(c->v, !nl, opts(c), c->ffd, fp32, s, gate);
    (void)hipEventRecord(e[1], s);
    (void)hipEventRecord(e[2], s);
    launch_scan(c->v, s, gate);
    (void)hipEventRecord(e[3], s);
    (void)hipEventRecord(e[4], s);
    launch_scatter(c->v, s, gate);
    (void)hipEventRecord(e[5], s);
    (void)hipEventRecord(e[6], s);
    launch_rank_payload(c->v, fp32, s, gate);
    (void)hipEventRecord(e[7], s);
    (void)hipEventRecord(e[14], s);
    if (nl) launch_nl_build(c->v, c->ffd, fp32, c->lj_kernel, s, gate);
    (void)hipEventRecord(e[15], s);
    (void)hipEventRecord(e[8], s);
    if (nl)
      launch_lj_nl(c->v, c->ffd, fp32, c->lj_kernel, last, c->homes, s);
    else
      launch_lj(c->v, c->ffd, fp32, c->lj_kernel, last, c->homes, s);
    (void)hipEventRecord(e[9], s);
    (void)hipEventRecord(e[10], s);
    launch_bonded(c->v, c->ffd, fp32, bonded_mode(c, true), last, c->remove_com != 0, c->dt, s);
    (void)hipEventRecord(e[11], s);
    (void)hipEventRecord(e[12], s);
    launch_reduce(c->v, last, true, opts(c), s);
    (void)hipEventRecord(e[13], s);
    advance_build_counter(c, forced);
  }
  launch_finalize(c->v, opts(c), s);
  c->step += n_steps;
  st = check_launch(c, "timed step");
  if (!st) st = hip_check(c, hipStreamSynchronize(s), "timed step sync");
  if (!st)
    for (int32_t k = 0; k < n_steps; ++k)
      for (int p = 0; p < P; ++p) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[((size_t)k * P + p) * 2], ev[((size_t)k * P + p) * 2 + 1]);
        ms_out[p] += ms;
      }
  for (auto& x : ev) (void)hipEventDestroy(x);
  return st;
}

md_status md_energies(md_ctx* c, md_energy* out) {
  if (!c || !out) return MD_ERR_ARG;
  if (taken_over(c)) return MD_ERR_STATE;
  md_status st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return st;
  std::vector<double> e((size_t)kEnergySlots * c->n_boxes);
  int32_t err = 0;
  if ((st = hip_check(c, hipMemcpy(e.data(), c->v.energy, 8 * e.size(), hipMemcpyDeviceToHost), "read energies")))
    return st;
  if ((st = hip_check(c, hipMemcpy(&err, c->v.err, 4, hipMemcpyDeviceToHost), "read error word"))) return st;
  for (int b = 0; b < c->n_boxes; ++b) {
    const double* q = &e[(size_t)kEnergySlots * b];
    out[b].e_lj = q[0];
    out[b].e_lj_shifted = q[1];
    out[b].e_bond = q[2];
    out[b].e_angle = q[3];
    out[b].e_dih = q[4];
    out[b].e_kin = q[5];
    out[b].temperature = q[6];
    out[b].virial = q[7];
    out[b].step = c->step;
    out[b].nh_xi = q[8];
    out[b].e_thermostat = q[9];
  }
  if (err & kErrNonFinite) {
    c->failed = true;
    return fail(c, MD_ERR_NONFINITE, "a position became non-finite");
  }
  return MD_OK;
}

md_status md_bins(md_ctx* c, const int32_t** cell_start, const int32_t** cell_atoms, int64_t* n_cells) {
  if (!c || !cell_start || !cell_atoms || !n_cells) return MD_ERR_ARG;
  if (taken_over(c)) return MD_ERR_STATE;
  *cell_start = c->v.cell_start;
  *cell_atoms = c->v.cell_atoms;
  *n_cells = c->v.C;
  return MD_OK;
}

md_status md_grid(const md_ctx* c, int32_t box, int32_t M[3], int64_t* cell_offset, int64_t* atom_offset) {
  if (!c || !M || box < 0 || box >= c->n_boxes) return MD_ERR_ARG;
  const BoxDev& B = c->hboxes[box];
  for (int d = 0; d < 3; ++d) M[d] = B.M[d];
  if (cell_offset) *cell_offset = B.cell_off;
  if (atom_offset) *atom_offset = B.atom_off;
  return MD_OK;
}

md_status md_forces(md_ctx* c, const void** f, int32_t* is_fp32) {
  if (!c || !f || !is_fp32) return MD_ERR_ARG;
  if (taken_over(c)) return MD_ERR_STATE;
  *f = c->v.f_tot;
  *is_fp32 = c->prec == MD_PREC_MIXED;
  return MD_OK;
}

md_status md_forces_lj(md_ctx* c, const void** f, int32_t* is_fp32) {
  if (!c || !f || !is_fp32) return MD_ERR_ARG;
  if (taken_over(c)) return MD_ERR_STATE;
  *f = c->v.f_lj;
  *is_fp32 = c->prec == MD_PREC_MIXED;
  return MD_OK;
}

md_status md_tuning(const md_ctx* c, int32_t* cell_div, int32_t* lj_kernel, int32_t* tile_homes) {
  if (!c || !cell_div || !lj_kernel) return MD_ERR_ARG;
  *cell_div = c->R;
  *lj_kernel = c->lj_kernel;
  if (tile_homes) *tile_homes = c->homes;
  return MD_OK;
}

md_status md_observables(md_ctx* c, const md_obs_config* o, uint64_t* pairs, uint64_t* dih, double* shape) {
  static_assert(kMaxObsBins == MD_OBS_MAX_BINS, "observable bins");
  if (!c || !o) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  if (pairs && (o->rdf_bins < 1 || o->rdf_bins > kMaxObsBins || !(o->rdf_rmax > 0.0) || !(o->rdf_rmax <= c->ff.rc)))
    return fail(c, MD_ERR_ARG, "rdf_bins must be 1..MD_OBS_MAX_BINS and 0 < rdf_rmax <= rc");
  if (dih && (o->dih_bins < 0 || o->dih_bins > kMaxObsBins - 3))
    return fail(c, MD_ERR_ARG, "dih_bins must be 0..MD_OBS_MAX_BINS - 3");
  const double dr = pairs ? o->rdf_rmax / o->rdf_bins : 0.0;
  for (int b = 0; b < c->n_boxes; ++b) {
    const int64_t n = (int64_t)c->n_chains[b] * c->chain_len;
    if (pairs)
      launch_obs_pairs(c->v, b, n, c->chain_len, c->ff.excl_depth, dr, o->rdf_bins,
                       (unsigned long long*)pairs + (int64_t)b * o->rdf_bins, c->stream);
    if (dih)
      launch_obs_dihedrals(c->v, b, n, c->chain_len, o->dih_bins,
                           (unsigned long long*)dih + (int64_t)b * (o->dih_bins + 3), c->stream);
    if (shape) launch_obs_chains(c->v, c->ffd, b, c->n_chains[b], c->chain_len, shape, c->stream);
  }
  return check_launch(c, "observables");
}

md_status md_ree_reference(md_ctx* c) {
  if (!c) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  enqueue_ree(c, true, nullptr);
  return check_launch(c, "end-to-end reference");
}

md_status md_ree_acf(md_ctx* c, double* acf) {
  if (!c || !acf) return MD_ERR_ARG;
  if (!usable(c)) return MD_ERR_STATE;
  enqueue_ree(c, false, acf);
  return check_launch(c, "end-to-end autocorrelation");
}

md_status md_list_builds(md_ctx* c, int64_t* builds) {
  if (!c || !builds) return MD_ERR_ARG;
  if (taken_over(c)) return MD_ERR_STATE;
  *builds = 0;
  if (!nl_mode(c)) return MD_OK;
  md_status st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return st;
  unsigned long long n = 0;
  if ((st = hip_check(c, hipMemcpy(&n, c->v.nl_builds, 8, hipMemcpyDeviceToHost), "read list builds"))) return st;
  *builds = (int64_t)n;
  return MD_OK;
}

md_status md_destroy(md_ctx* c) {
  if (!c) return MD_ERR_ARG;
  (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return MD_OK;
}

const char* md_status_string(md_status s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_ERR_ARG: return "invalid argument";
    case MD_ERR_BOX_TOO_SMALL: return "box too small for the cell stencil";
    case MD_ERR_NONFINITE: return "non-finite position or force";
    case MD_ERR_WORKSPACE: return "workspace too small or misaligned";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_STATE: return "context in error state";
    case MD_ERR_NLIST: return "neighbour list invalid (not returned: lists rebuild on displacement)";
  }
  return "unknown status";
}

const char* md_last_error(const md_ctx* c) { return c ? c->last_error.c_str() : ""; }

}  // extern "C"
