/* oracle_md.h -- FP64 CPU reference for the per-timestep path of united-atom
 * polyethylene molecular dynamics (Xu et al., "Molecular Dynamics Simulation of
 * Macromolecules Using Graphics Processing Unit").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares no
 * code, header, table or helper with it.
 *
 * It computes, plainly and slowly, in double precision:
 *   - the wrap of positions into the periodic box and the cell index of each atom
 *     (Section 3.1: grid of cells with edge at least the cutoff);
 *   - the counting sort of atoms into cells (Section 3.1, the binning step);
 *   - the truncated Lennard-Jones force, energy and virial (Eq. 2; Section 3.2),
 *     both by brute force over all pairs and by the paper's grid search over the
 *     neighbouring cells, with only 1-2 and 1-3 chain neighbours excluded
 *     (Section 3.1, Dreiding II);
 *   - bond, angle and dihedral forces and energies (Eqs. 4-6; Section 3.3);
 *   - one velocity-Verlet step with optional Berendsen scaling (Section 3.4
 *     integrates with leap-frog, whose positions are the same);
 *   - one leap-frog step with the Nose-Hoover thermostat (Section 3 opening and
 *     Section 3.4: leap-frog, NVT through the Nose-Hoover extended system);
 *   - removal of each box's centre-of-mass velocity (Section 3 opening and the
 *     COM-removal timing of Section 4; translation only, see ora_integ);
 *   - the structural observables of Section 5: the pair-distance histogram behind the
 *     radial distribution function (Fig. 10), the dihedral (conformation) distribution
 *     and trans fraction (Figs. 9, 15), per-chain radius of gyration and end-to-end
 *     vector (Figs. 8, 12), and the autocorrelation of the end-to-end vectors (Fig. 8).
 *
 * Units: Angstrom, fs, g/mol, kcal/mol, K.  Every array is caller-owned host
 * memory; coordinates are structure-of-arrays.  Functions return 0 on success and
 * a negative value on bad arguments.  Nothing here allocates memory that outlives
 * a call.
 */
#ifndef ORACLE_MD_H
#define ORACLE_MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double mass[2];      /* g/mol; type 0 = CH2 (C_32), 1 = CH3 (C_33) */
  double sigma[2];     /* A */
  double epsilon[2];   /* kcal/mol */
  double kb, b0;       /* Eq. (4): kcal/mol/A^2, A */
  double ka, theta0_deg;  /* Eq. (5): kcal/mol/rad^2, degrees */
  double kphi, phis_deg;  /* Eq. (6): kcal/mol, degrees */
  int32_t n_dih;          /* Eq. (6) periodicity */
  double rc;              /* cutoff, A; pairs with r < rc interact */
  int32_t excl_depth;     /* pairs closer than this many bonds along a chain are excluded */
} ora_ff;

/* Energies and virial of one configuration. */
typedef struct {
  double e_lj, e_lj_shifted, e_bond, e_angle, e_dih, virial_lj, virial_bonded;
} ora_energy;

int ora_set_threads(int n);   /* OpenMP threads for the per-atom loops; returns threads in use */

/* Wrap each coordinate into [0, L_d) in place: if outside, s = floor(x * invL),
   x = fma(-s, L, x), then one correction by L each way.  invL = 1/L. */
int ora_wrap(int64_t n, double* x, double* y, double* z, const double L[3]);

/* Cell index per atom: k_d = clamp(floor(x_d * (M_d / L_d)), 0, M_d - 1),
   cell = k_x + M_x * (k_y + M_y * k_z). */
int ora_cell_index(int64_t n, const double* x, const double* y, const double* z,
                   const double L[3], const int32_t M[3], int32_t* cell);

/* Counting sort: cnt[c] atoms per cell, cell_start = exclusive prefix sum of cnt
   (n_cells + 1 entries), cell_atoms lists atoms of each cell in ascending index. */
int ora_bin(int64_t n, const int32_t* cell, int64_t n_cells, int32_t* cnt, int32_t* cell_start,
            int32_t* cell_atoms);

/* Lennard-Jones by brute force over all unordered pairs (minimum image).
   Forces are written (not accumulated). */
int ora_lj_brute(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                 const double* z, const uint8_t* type, const double L[3], double* fx, double* fy,
                 double* fz, ora_energy* e);

/* Lennard-Jones by the grid search: each atom visits the (2R+1)^3 cells around its
   own (R = stencil radius, M_d >= 2R+1, L_d / M_d >= rc / R), every pair from both
   sides.  If `subset` is non-null only atoms subset[0..n_subset) get forces (others
   are left untouched) and e may be null. */
int ora_lj_cells(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                 const double* z, const uint8_t* type, const double L[3], const int32_t M[3],
                 int32_t R, const int64_t* subset, int64_t n_subset, double* fx, double* fy,
                 double* fz, ora_energy* e);

/* Bond, angle and dihedral terms of linear chains of chain_len atoms (atom c*chain_len+p
   is site p of chain c).  Forces are ADDED to fx, fy, fz. */
int ora_bonded(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
               const double* z, const double L[3], double* fx, double* fy, double* fz,
               ora_energy* e);

/* The bonded terms of one chain as the oracle enumerates them: k = 2 (bonds),
   3 (angles), 4 (dihedrals); writes up to max_terms tuples of k 0-based site indices
   to out and returns the number of terms. */
int ora_chain_terms(int32_t chain_len, int32_t k, int32_t* out, int32_t max_terms);

/* Single-term helpers on explicit coordinates (no periodicity); forces written to f[3*k]. */
double ora_bond_term(const ora_ff* ff, const double* xi, const double* xj, double* f);
double ora_angle_term(const ora_ff* ff, const double* xi, const double* xj, const double* xk,
                      double* f, double* theta_out);
double ora_dihedral_term(const ora_ff* ff, const double* xi, const double* xj, const double* xk,
                         const double* xl, double* f, double* phi_out);

/* Total force (LJ by grid search with stencil radius R, plus bonded). */
int ora_forces(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
               const double* z, const uint8_t* type, const double L[3], const int32_t M[3],
               int32_t R, double* fx, double* fy, double* fz, ora_energy* e);

/* Compensated (Neumaier) sum of v[0..n) in index order. */
double ora_sum(int64_t n, const double* v);

/* Kinetic energy (kcal/mol) and temperature (K, 3N-3 degrees of freedom). */
int ora_kinetic(const ora_ff* ff, int64_t n, const double* vx, const double* vy, const double* vz,
                const uint8_t* type, double* ke, double* temperature);

typedef struct {
  double dt;     /* fs */
  double tau;    /* fs: Berendsen coupling time (ora_run), Nose-Hoover period tau_T (ora_run_leapfrog) */
  double T0;     /* K; <= 0 disables the thermostat (NVE) */
  int32_t remove_com;  /* 1: after every step subtract the centre-of-mass velocity,
                          u = sum m v / sum m, from every velocity (translation only; a
                          rotation of a periodic box is not a conserved motion) */
} ora_integ;

/* Centre-of-mass velocity u = sum_i m_i v_i / sum_i m_i (compensated sums, index order). */
int ora_com_velocity(const ora_ff* ff, int64_t n, const double* vx, const double* vy, const double* vz,
                     const uint8_t* type, double u[3]);

/* Nose-Hoover state: friction xi (1/fs), its time integral eta, and (output) the energy
   of the extended variables, dof R T0 (xi^2 / (2 omega^2) + eta), omega = 2 pi / tau. */
typedef struct {
  double xi, eta, e_thermostat;
} ora_nh;

/* n_steps of velocity Verlet on one box.  On entry f holds the total force at x;
   on exit x, v and f are advanced.  Per step: v += dt/2 a; x += dt v; wrap;
   f = F(x); v += dt/2 a; [remove_com: v -= u]; KE, T; if T0 > 0, v *= lambda with
   lambda = sqrt(1 + dt/tau (T0/T - 1)).  e_out / ke_out / t_out (may be null) get
   the energies of the last step (kinetic energy and temperature before scaling). */
int ora_run(const ora_ff* ff, const ora_integ* in, int64_t n, int32_t chain_len, double* x,
            double* y, double* z, double* vx, double* vy, double* vz, double* fx, double* fy,
            double* fz, const uint8_t* type, const double L[3], const int32_t M[3], int32_t R,
            int32_t n_steps, ora_energy* e_out, double* ke_out, double* t_out);

/* n_steps of leap-frog with the Nose-Hoover thermostat on one box.  Equations of motion:
   dx/dt = v, dv/dt = F/m - xi v, dxi/dt = omega^2 (T/T0 - 1), deta/dt = xi, with
   omega = 2 pi / tau (thermostat mass Q = tau^2 T0 / (4 pi^2) per unit dof R).
   v holds half-step velocities: on entry v(t - dt/2) with f = F(x(t)).  Per step:
     v <- ((1 - dt/2 xi) v + dt a) / (1 + dt/2 xi)      (friction at mid-interval)
     x <- wrap(x + dt v);  f = F(x)
     [remove_com: v <- v - u]
     KE, T of v (the half-step velocities);
     if T0 > 0: xi' = xi + dt omega^2 (T/T0 - 1); eta <- eta + dt (xi + xi')/2; xi <- xi'.
   nh (may be null: start from rest, state discarded) carries xi and eta across calls.
   Outputs as ora_run. */
int ora_run_leapfrog(const ora_ff* ff, const ora_integ* in, ora_nh* nh, int64_t n, int32_t chain_len,
                     double* x, double* y, double* z, double* vx, double* vy, double* vz, double* fx,
                     double* fy, double* fz, const uint8_t* type, const double L[3], const int32_t M[3],
                     int32_t R, int32_t n_steps, ora_energy* e_out, double* ke_out, double* t_out);

/* Pair-distance histogram (Section 5, Fig. 10): every unordered pair i < j that the force
   field does not exclude (excluded: same chain, at most excl_depth bonds apart), with the
   minimum-image distance r < rmax, counted in bin k = floor(r / dr), dr = rmax / n_bins.
   The bin is decided on r^2 = dx*dx + dy*dy + dz*dz (FP64, in that order, no fused
   multiply-add) against the squared edges (k * dr)^2, so no square root takes part in it.
   M == NULL: all pairs by brute force.  Otherwise the grid search over the 27 cells around
   each atom's cell (M[d] >= 3, L[d] / M[d] >= rmax; positions wrapped).  counts[n_bins]
   are written. */
int ora_pair_histogram(int64_t n, int32_t chain_len, int32_t excl_depth, const double* x, const double* y,
                       const double* z, const double L[3], const int32_t* M, double rmax, int32_t n_bins,
                       uint64_t* counts);

/* Dihedral statistics (Section 5, Figs. 9 and 15): the IUPAC angle phi in (-pi, pi] of every
   dihedral of every chain (bonds minimum-imaged; the angle as ora_dihedral_term computes
   it).  hist[k] counts k = floor((phi + pi) * (n_bins / (2 pi))), clamped to n_bins - 1
   (n_bins may be 0: no histogram); classes[0] = trans (|phi| > 2 pi / 3), classes[1] =
   gauche+ (0 <= phi <= 2 pi / 3), classes[2] = gauche- (-2 pi / 3 <= phi < 0). */
int ora_dihedral_stats(int64_t n, int32_t chain_len, const double* x, const double* y, const double* z,
                       const double L[3], int32_t n_bins, uint64_t* hist, uint64_t classes[3]);

/* Chain shape (Section 5, Figs. 8 and 12): each chain unwrapped link by link from its first
   atom (u_0 = x_0, u_{p+1} = u_p + minimum image of x_{p+1} - x_p), the mass-weighted
   radius of gyration Rg^2 = sum m |u - u_cm|^2 / sum m with u_cm = sum m u / sum m, and the
   end-to-end vector u_last - u_first.  out[4 c] = Rg^2 (A^2), out[4 c + 1..3] = R_ee (A). */
int ora_chain_shape(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                    const double* z, const uint8_t* type, const double L[3], double* out);

/* End-to-end vector autocorrelation (Section 5, Fig. 8): the normalised correlation of each
   chain's end-to-end vector with its value at a reference time, averaged over the chains,
   acf = sum_c R_c(t) . R_c(0) / sum_c |R_c(0)|^2.  Each R is the sum of the chain's
   minimum-imaged bond vectors, first atom to last (as ora_chain_shape); the two sums are
   compensated.  (x0, y0, z0): positions at the reference time; (x, y, z): at time t.
   *acf is written. */
int ora_ree_acf(int64_t n, int32_t chain_len, const double* x0, const double* y0, const double* z0,
                const double* x, const double* y, const double* z, const double L[3], double* acf);

#ifdef __cplusplus
}
#endif
#endif
