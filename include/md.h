/* md.h -- C ABI of the MI355X (gfx950) library for the per-timestep hot path of
 * united-atom polyethylene molecular dynamics, after Xu, Ren, Ge, Yu, Yang, Li,
 * "Molecular Dynamics Simulation of Macromolecules Using Graphics Processing Unit".
 *
 * One time step, all on the GPU (Section 3, Figure 1):
 *   - bin rebuild (Section 3.1): wrap positions into the periodic box, cell index per
 *     atom, count per cell, exclusive scan, stable scatter into cell lists, and a
 *     sorted coordinate payload for the force kernel;
 *   - non-bonded force (Section 3.2, Eq. 2): truncated Lennard-Jones over the cells
 *     around each atom's cell, excluding only 1-2 and 1-3 chain neighbours;
 *   - bonded forces (Section 3.3, Eqs. 3-6): bond, angle and dihedral terms of the
 *     linear chains;
 *   - update (Section 3.4): velocity Verlet (the same positions as the paper's
 *     leap-frog) with optional Berendsen velocity scaling, or the paper's leap-frog with
 *     the Nose-Hoover thermostat; optional removal of each box's centre-of-mass velocity
 *     (Section 3); per-box kinetic energy, potential energies and virial summed in
 *     compensated double precision.
 *
 * Units: Angstrom, fs, g/mol, kcal/mol, K.
 *
 * Memory.  The library allocates no device memory.  Positions, velocities, types
 * and one workspace are caller-owned device buffers (for instance torch tensors);
 * they must outlive the context, which keeps non-owning pointers.  Coordinates are
 * structure-of-arrays: pos[0..N) = x, pos[N..2N) = y, pos[2N..3N) = z, FP64.
 * Several independent periodic boxes may be simulated at once ("batched"): box b
 * owns the contiguous atoms [atom_offset(b), atom_offset(b) + n_chains[b] * chain_len),
 * and its chains are contiguous runs of chain_len atoms; atom c*chain_len + p is
 * site p of chain c (0-based; the paper's indices are 1-based).
 *
 * Streams.  Every call enqueues work on the HIP stream given at init and returns
 * without waiting, except md_energies, md_tuning and md_destroy, which synchronise
 * that stream.  Calls on one context must not overlap from several host threads.
 *
 * Errors.  Every function returns md_status and never throws.  Argument errors are
 * detected on the host before anything is enqueued.  Errors found on the device
 * (non-finite positions or forces) set a sticky device word that the next
 * md_energies reports; the context then refuses md_step until re-initialised.
 *
 * Range of the mixed form.  Coordinates are held relative to their cell centre as int32
 * fixed point (2^-25 A), so the configuration must keep (R + 2) * cell edge + nl_skin below
 * 63 A on every box and axis (R the stencil radius; the LJ kernels shift candidates by up to
 * R + 1 edges); md_workspace_bytes and md_init_system refuse it otherwise (MD_ERR_ARG).  Atom
 * types are 0 or 1 (Table I's two united atoms).
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MD_OK = 0,
  MD_ERR_ARG = -1,            /* null pointer, bad size or inconsistent configuration */
  MD_ERR_BOX_TOO_SMALL = -2,  /* a box has fewer than 2R+1 cells along a dimension */
  MD_ERR_NONFINITE = -3,      /* a coordinate or force became NaN or infinite (device) */
  MD_ERR_WORKSPACE = -4,      /* workspace smaller than md_workspace_bytes, or misaligned */
  MD_ERR_HIP = -6,            /* a HIP runtime call failed; md_last_error has the text */
  MD_ERR_STATE = -7,          /* the context is in an error state; re-initialise it */
  MD_ERR_NLIST = -8           /* reserved; not returned by this version: neighbour lists are rebuilt
                                 in the same step as soon as an atom has moved more than half the
                                 skin, and a cell or atom whose list outgrew its capacity walks its
                                 stencil instead, so a list never misses a pair */
} md_status;

typedef enum {
  MD_PREC_FP64 = 0,   /* every force, energy and state update in double precision */
  MD_PREC_MIXED = 1   /* pair and bonded forces in FP32 with FP32 per-atom accumulation (pairs
                         closer than 0.75 sigma, and pairs whose side of the cutoff FP32 cannot
                         tell, are decided and evaluated in FP64); positions, velocities and the
                         update in FP64; energy and virial sums in compensated FP64 */
} md_precision;

typedef enum {
  MD_LJ_AUTO = 0,       /* chosen by the autotuner at init */
  MD_LJ_ATOM = 1,       /* one lane per home atom walking the neighbouring cells */
  MD_LJ_CELLTILE = 2,   /* one wavefront per home cell: home atoms wave-uniform, candidate
                           atoms across the lanes */
  MD_LJ_CELLTILE_NB = 3, /* as MD_LJ_CELLTILE, with the pair force evaluated on every lane and
                            zeroed outside the cutoff instead of branching (mixed precision) */
  MD_LJ_NLIST = 4,       /* neighbour-list mode (nl_skin > 0): a Verlet list per atom, one lane
                            per atom walking it */
  MD_LJ_NLIST_TILE = 5,  /* neighbour-list mode: a list per cell (every atom within rc + skin of
                            any atom of the cell at the build), streamed by the cell-tile kernel
                            against the cell's atoms */
  MD_LJ_HALFSHELL = 6    /* cell path, opt-in (never chosen by the autotuner): each pair evaluated
                            once (Newton's third law; the paper's Section 4.2 names the doubled
                            pair work of its per-atom kernels as a cost), both forces
                            added to int64 fixed-point accumulators with device atomics, so the
                            sums are exact and order-independent.  Measured slower than the full
                            shell on this device: the atomics cost more than the second
                            evaluation they save */
} md_lj_kernel;

typedef enum {
  MD_INT_VERLET_BERENDSEN = 0, /* velocity Verlet; with T0 > 0, Berendsen scaling
                                  v <- lambda v, lambda = sqrt(1 + dt/tau (T0/T - 1)), T from the
                                  full-step velocities */
  MD_INT_LEAPFROG_NH = 1       /* leap-frog with the Nose-Hoover thermostat (Section 3.4):
                                  dv/dt = F/m - xi v, dxi/dt = omega^2 (T/T0 - 1), omega = 2 pi / tau.
                                  Velocities are half-step velocities: the ones passed to init are
                                  v(-dt/2), and after n steps vel holds v((n - 1/2) dt).  Per step:
                                  v <- ((1 - dt xi/2) v + dt a) / (1 + dt xi/2); x <- x + dt v;
                                  forces; [COM removal]; T from v; xi advanced with that T.
                                  xi starts at 0; with T0 <= 0 it stays 0 (NVE leap-frog) */
} md_integrator;

/* Force field (Table I, Eqs. 2-6).  Types: 0 = CH2 (C_32), 1 = CH3 (C_33).  LJ pair
   parameters follow Lorentz-Berthelot mixing. */
typedef struct {
  double mass[2];         /* g/mol */
  double sigma[2];        /* A */
  double epsilon[2];      /* kcal/mol */
  double kb, b0;          /* Eq. (4): E = kb/2 (r - b0)^2; kcal/mol/A^2, A */
  double ka, theta0_deg;  /* Eq. (5): E = ka/2 (theta - theta0)^2; kcal/mol/rad^2, deg */
  double kphi, phis_deg;  /* Eq. (6): E = kphi (1 + cos(n phi - phis)); kcal/mol, deg; */
  int32_t n_dih;          /*   phi is IUPAC (trans = 180 deg), n >= 1 */
  double rc;              /* cutoff, A: a pair interacts iff r < rc */
  int32_t excl_depth;     /* pairs at most this many bonds apart on a chain are excluded
                             (2 = the 1-2 and 1-3 exclusions of Dreiding II, Section 3.1) */
} md_forcefield;

typedef struct {
  int32_t n_boxes;            /* >= 1 */
  int32_t chain_len;          /* atoms per chain, >= 4 */
  const int32_t* n_chains;    /* host [n_boxes], >= 1 each */
  const double* box;          /* host [n_boxes * 3], box edges in A */
  const double* T0;           /* host [n_boxes], thermostat target in K; <= 0: NVE */
  double dt_fs;               /* time step, fs (> 0) */
  double tau_fs;              /* thermostat time, fs (> 0): Berendsen coupling time, or the
                                 Nose-Hoover period tau_T (thermostat mass tau_T^2 T0 / (4 pi^2)
                                 per degree of freedom and unit gas constant) */
  int32_t precision;          /* md_precision */
  int32_t cell_div;           /* R: cells of edge >= rc / R, (2R+1)^3 cells visited;
                                 1 = the paper's grid (edge >= cutoff), 2 = half cells;
                                 0 = chosen by the autotuner at init */
  int32_t lj_kernel;          /* md_lj_kernel: 1..3 or 6 (cell path) or 4..5 (neighbour-list mode),
                                 or 0 for the autotuner (which never picks 6) */
  int32_t use_graph;          /* 1: md_step replays a captured hipGraph of the step */
  double nl_skin;             /* > 0: neighbour-list mode, the paper's force path (Sections 3.1-3.2).
                                 A Verlet list of the pairs closer than rc + nl_skin (A) is built
                                 from the bins.  Every step checks each atom's displacement since
                                 the last build; when one exceeds nl_skin / 2 the bins and the list
                                 are rebuilt in that step, before the forces (a device flag gates
                                 the rebuild kernels, so graph replay needs no host decision).
                                 0: forces from the cells every step */
  int32_t nl_every;           /* neighbour-list mode: >= 1 also rebuilds every nl_every steps
                                 (the paper rebuilds every 10), 0 only on displacement */
  int32_t integrator;         /* md_integrator */
  int32_t remove_com;         /* 1: after every step subtract each box's centre-of-mass velocity
                                 sum(m v) / sum(m) (after the drift, before the thermostat reads
                                 T; translation only: a periodic box has no conserved rotation);
                                 the reported kinetic energy is then that of the motion relative
                                 to the centre of mass.  0: no removal */
  int32_t tile_homes;         /* home atoms each wavefront of the mixed cell-tile kernels (2, 3, 5)
                                 holds at a time against its stream of candidates: 4, 8 or 16;
                                 0 = 8, or the autotuner's choice when it runs (cell_div = 0 or
                                 lj_kernel = 0) */
} md_config;

/* Per-box results of the most recent energy evaluation. */
typedef struct {
  double e_lj;           /* truncated LJ energy, kcal/mol */
  double e_lj_shifted;   /* sum over counted pairs of E(r) - E(rc) (reporting only) */
  double e_bond, e_angle, e_dih;
  double e_kin;          /* kinetic energy, kcal/mol: velocity Verlet, of the full-step velocities
                            before Berendsen scaling; leap-frog, of the half-step velocities */
  double temperature;    /* K, 3N - 3 degrees of freedom */
  double virial;         /* sum over interactions of r . F (LJ + bonded), kcal/mol */
  int64_t step;          /* steps taken since init */
  double nh_xi;          /* Nose-Hoover friction xi for the next step, 1/fs (0 otherwise) */
  double e_thermostat;   /* Nose-Hoover extended-system energy dof R T0 (xi^2 / (2 omega^2) + eta),
                            eta = time integral of xi, kcal/mol; KE + PE + e_thermostat is
                            conserved (0 for velocity Verlet) */
} md_energy;

typedef struct md_ctx md_ctx;

/* Input of initial conditions (Fig. 1): bytes of device workspace the configuration needs
   (for cell_div = 0 or lj_kernel = 0, the largest over the autotuner's candidates).  Never
   fails for a valid configuration; MD_ERR_ARG (including a mixed configuration outside the
   fixed-point range) / MD_ERR_BOX_TOO_SMALL (fewer than 2R + 1 cells of edge >= rc / R on an
   axis for every stencil radius R) otherwise. */
md_status md_workspace_bytes(const md_forcefield* ff, const md_config* cfg, size_t* bytes);

/* Input of initial conditions (Fig. 1; positions, velocities, types and the chain topology of
   Section 2): validates the configuration, copies the small per-box tables to the device,
   builds the bins and computes the forces at the initial positions (so the first
   half-kick has a force), stores the end-to-end vectors as the autocorrelation's reference,
   and, when use_graph = 1, captures the step graph.  MD_ERR_ARG also for an atom type
   other than 0 or 1 (read from the device type array).
   pos, vel: device FP64 [3 * N], updated in place by md_step.
   type:     device uint8 [N], 0 or 1.
   workspace: device, >= md_workspace_bytes, 256-byte aligned.
   stream:   a hipStream_t (null = the default stream).
   With cell_div = 0 or lj_kernel = 0 the autotuner times the candidates on these
   inputs first (positions are not changed by it).  On success *out is a new context. */
md_status md_init_system(const md_forcefield* ff, const md_config* cfg, double* pos, double* vel,
                         const uint8_t* type, void* workspace, size_t ws_bytes, void* stream,
                         md_ctx** out);

/* Allocation-free set-up, for callers that cannot allocate device memory (code that must not
   call hipMalloc or an allocating library routine: serving loops, harnesses that forbid it).
   As md_init_system, except that the workspace is a device array inside the library,
   MD_STATIC_WORKSPACE_BYTES per GPU (allocated when the library's code object is loaded on that
   GPU and held until the process ends), so the caller passes only the positions, velocities
   and types.  Nothing is allocated on the device by this call or by later calls on the context.
   Restrictions: use_graph = 0 (instantiating a graph allocates), and cell_div and lj_kernel
   given (nonzero: the autotuner's timing is not used).  Errors: MD_ERR_ARG for those, as
   md_init_system otherwise; MD_ERR_WORKSPACE when md_workspace_bytes exceeds
   MD_STATIC_WORKSPACE_BYTES (nothing is enqueued then); MD_ERR_HIP if the array's device address
   cannot be obtained.
   Sharing: every allocation-free context on one GPU uses that GPU's one array.  A call takes it
   over: afterwards every call on an older allocation-free context of the same GPU returns
   MD_ERR_STATE (destroy it; only md_destroy, md_grid, md_tuning and md_last_error still work).
   The array keeps the last context's contents; the set-up clears everything that must start at
   zero.  Calls on two contexts that share the array race if they overlap in time (for instance
   on two streams); contexts made by md_init_system are unaffected. */
#define MD_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
md_status md_init_system_static(const md_forcefield* ff, const md_config* cfg, double* pos, double* vel,
                                const uint8_t* type, void* stream, md_ctx** out);

/* Binning (Section 3.1): wrap positions into their box, recompute cell indices and rebuild
   the cell lists and the sorted coordinate payload; in neighbour-list mode also rebuild the
   list.  Enqueues only. */
md_status md_rebuild_bins(md_ctx* ctx);

/* Forces (Sections 3.2-3.3): at the positions of the last bin rebuild (in neighbour-list
   mode, the current positions through the list), LJ (Eq. 2) plus bonded (Eqs. 4-6);
   with_energy != 0 also evaluates the per-box energies and virial (read them with
   md_energies).  Enqueues only. */
md_status md_compute_forces(md_ctx* ctx, int32_t with_energy);

/* The MD loop (Section 3.4, Fig. 1): advance every box by n_steps (>= 0) steps of the
   configured integrator with the bins rebuilt every step (in neighbour-list mode: when an atom
   has moved more than half the skin, or every nl_every steps, together with the list);
   energies are evaluated on the last step.  Enqueues only. */
md_status md_step(md_ctx* ctx, int32_t n_steps);

/* Phases timed by md_step_timed. */
enum {
  MD_PHASE_INTEGRATE_BIN = 0,  /* velocity update (pending Berendsen factor and COM velocity,
                                  half kick, or the leap-frog kick), drift, wrap, cell index, count */
  MD_PHASE_SCAN = 1,           /* exclusive scan of the cell counts */
  MD_PHASE_SCATTER = 2,        /* unordered cell lists */
  MD_PHASE_RANK = 3,           /* ordered cell lists and the sorted payload */
  MD_PHASE_LJ = 4,             /* Lennard-Jones forces */
  MD_PHASE_BONDED = 5,         /* bonded forces, total force, second half kick (velocity Verlet),
                                  kinetic energy and momentum partial sums */
  MD_PHASE_REDUCE = 6,         /* per-box sums, the thermostat and the COM velocity */
  MD_PHASE_NLIST = 7,          /* neighbour-list build (neighbour-list mode, build steps only) */
  MD_N_PHASES = 8
};
/* In neighbour-list mode MD_PHASE_INTEGRATE_BIN covers the update, the displacement
   check and the payload refresh on the steps between builds, and the scan, scatter,
   rank and list phases are empty on those steps. */

/* Measurement of the MD loop (Section 4's per-kernel timings): the same as md_step but
   launched without the graph and with a pair of HIP events around every phase on the
   context's stream; adds each phase's summed duration in milliseconds to
   ms_out[MD_N_PHASES].  Synchronises the stream before returning. */
md_status md_step_timed(md_ctx* ctx, int32_t n_steps, double* ms_out);

/* Output of the step's energies (Section 3.4: kinetic energy and temperature; Eqs. 2, 4-6:
   the potential energies; the virial): synchronises the stream and copies the per-box results
   to out_host[n_boxes] (host).  Returns MD_ERR_NONFINITE if the device flagged a non-finite
   value (sticky: the context then refuses further steps), MD_ERR_STATE for an
   allocation-free context whose array was taken over, MD_ERR_HIP if a copy fails. */
md_status md_energies(md_ctx* ctx, md_energy* out_host);

/* The bins of Section 3.1 (the paper's cell table, here in compressed form): device views of
   the cell lists of the last rebuild, cell_start[n_cells + 1] (exclusive prefix sums, cells of
   all boxes concatenated box by box) and cell_atoms[N] (global atom indices, ascending within a
   cell).  Owned by the workspace; valid until the next rebuild. */
md_status md_bins(md_ctx* ctx, const int32_t** cell_start, const int32_t** cell_atoms,
                  int64_t* n_cells);

/* The grid of Section 3.1 for one box: cells per dimension (cell index = kx + M[0] * (ky +
   M[1] * kz)), and the offsets of its first cell and first atom in the concatenated arrays. */
md_status md_grid(const md_ctx* ctx, int32_t box, int32_t M[3], int64_t* cell_offset,
                  int64_t* atom_offset);

/* The force of Sections 3.2-3.3: device view of the total force of the last evaluation,
   SoA [3 * N], FP32 when *is_fp32 = 1 (mixed precision) else FP64; kcal/mol/A.  Owned by the
   workspace; valid until the next evaluation. */
md_status md_forces(md_ctx* ctx, const void** f, int32_t* is_fp32);

/* The Lennard-Jones part (Section 3.2, Eq. 2) of the force alone, same layout as md_forces. */
md_status md_forces_lj(md_ctx* ctx, const void** f, int32_t* is_fp32);

/* The cell size of Section 3.1 (edge >= rc / cell_div), the LJ kernel and the home atoms per
   cell-tile wavefront in use (what the autotuner chose, if asked; tile_homes may be null).
   Host only. */
md_status md_tuning(const md_ctx* ctx, int32_t* cell_div, int32_t* lj_kernel, int32_t* tile_homes);

/* Structural observables of Section 5 (Figs. 8-10, 12, 15). */
#define MD_OBS_MAX_BINS 2048
typedef struct {
  int32_t rdf_bins;    /* pair-distance bins over [0, rdf_rmax), 1..MD_OBS_MAX_BINS */
  double rdf_rmax;     /* A, 0 < rdf_rmax <= rc */
  int32_t dih_bins;    /* dihedral-angle bins over (-180, 180] deg, 0..MD_OBS_MAX_BINS - 3 */
} md_obs_config;

/* Observables of the current positions, per box, into caller-owned device buffers (any of
   the three may be null to skip that part):
   pair_counts     uint64 [n_boxes * rdf_bins]: unordered pairs the force field does not
                   exclude with minimum-image distance r < rdf_rmax, in bin floor(r / dr),
                   dr = rdf_rmax / rdf_bins.  The bin is decided in FP64 on r^2 against the
                   squared edges (k dr)^2, so the counts are exact.  g(r) of bin k is
                   counts[k] / (N (N - 1) / 2 * shell volume / V) (excluded pairs not removed
                   from the normalisation).
   dihedral_counts uint64 [n_boxes * (dih_bins + 3)]: per box, the histogram of the IUPAC
                   dihedral angle phi in (-pi, pi], bin floor((phi + pi) dih_bins / (2 pi)),
                   then the numbers of trans (|phi| > 120 deg), gauche+ (0 <= phi <= 120 deg)
                   and gauche- dihedrals.
   chain_shape     double [n_chains_total * 4]: per chain (box by box), the mass-weighted
                   R_g^2 (A^2) of the chain unwrapped bond by bond, and the end-to-end vector.
   Uses the cell lists of the last rebuild (current after md_step; in neighbour-list mode
   those of the last list build, which still cover every pair within rc).  Enqueues only. */
md_status md_observables(md_ctx* ctx, const md_obs_config* cfg, uint64_t* pair_counts,
                         uint64_t* dihedral_counts, double* chain_shape);

/* End-to-end vector autocorrelation (Section 5, Fig. 8).  md_ree_reference stores every
   chain's end-to-end vector (the sum of its minimum-imaged bonds, first atom to last) as the
   reference, time zero (md_init_system stores the initial ones).  md_ree_acf writes, per box,
   acf[b] = sum_c R_c . R_c(0) / sum_c |R_c(0)|^2 over the box's chains (acf: device double
   [n_boxes], caller-owned; sums in a fixed order, double-double).  Both enqueue only. */
md_status md_ree_reference(md_ctx* ctx);
md_status md_ree_acf(md_ctx* ctx, double* acf);

/* Neighbour-list mode: the number of list rebuilds the steps have made since init (those of
   md_init_system and md_rebuild_bins not counted), for monitoring the rebuild rate; 0 on the
   cell path.  Synchronises the stream. */
md_status md_list_builds(md_ctx* ctx, int64_t* builds);

/* Frees the host-side context and its graph; device buffers stay with the caller. */
md_status md_destroy(md_ctx* ctx);

const char* md_status_string(md_status s);
const char* md_last_error(const md_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
