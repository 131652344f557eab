/* oracle_md.c -- FP64 CPU reference (TEST INFRASTRUCTURE ONLY; see oracle_md.h).
 *
 * Plain C99, double precision, built with -O2 -ffp-contract=off (no fused
 * multiply-add except where fma() is written out).  Each function follows the
 * paper's definition directly:
 *   Eq. (2)  Lennard-Jones          E = 4 eps [(sigma/r)^12 - (sigma/r)^6], r < rc
 *   Eq. (4)  bond                   E = 1/2 kb (r - b)^2
 *   Eq. (5)  angle                  E = 1/2 ka (theta - theta0)^2
 *   Eq. (6)  dihedral               E = kphi (1 + cos(n phi - phi_s))
 *   Section 3.1  cells of edge >= cutoff, an atom searches its own and the
 *                neighbouring cells; 1-2 and 1-3 chain neighbours are excluded
 *   Section 3.4  time integration: velocity Verlet with Berendsen scaling, and the
 *                paper's leap-frog with the Nose-Hoover extended system
 *   Section 3    removal of the centre-of-mass velocity
 *   Section 5    pair-distance histogram, dihedral statistics, chain shape
 * The dihedral angle follows the IUPAC convention (trans = 180 deg), the reading under
 * which trans and gauche are minima of Eq. (6) with n = 3, phi_s = 0.
 */
#include "oracle_md.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* (kcal/mol/A) / (g/mol) in A/fs^2, and the gas constant in kcal/mol/K */
static const double ACC_UNIT = 4.184e-4;
static const double R_GAS = 1.987204259e-3;

int ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ---------- compensated summation (Neumaier) ---------- */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

double ora_sum(int64_t n, const double* v) {
  nsum a = {0, 0};
  for (int64_t i = 0; i < n; ++i) nadd(&a, v[i]);
  return nval(&a);
}

/* ---------- periodic helpers ---------- */
static double wrap1(double x, double L, double invL) {
  if (x >= 0.0 && x < L) return x;
  double s = floor(x * invL);
  double y = fma(-s, L, x);
  if (y >= L) y -= L;
  if (y < 0.0) y += L;
  return y;
}

static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

int ora_wrap(int64_t n, double* x, double* y, double* z, const double L[3]) {
  if (n < 0 || !L) return -1;
  double* c[3] = {x, y, z};
  for (int d = 0; d < 3; ++d) {
    double invL = 1.0 / L[d];
    for (int64_t i = 0; i < n; ++i) c[d][i] = wrap1(c[d][i], L[d], invL);
  }
  return 0;
}

int ora_cell_index(int64_t n, const double* x, const double* y, const double* z,
                   const double L[3], const int32_t M[3], int32_t* cell) {
  if (n < 0 || !L || !M) return -1;
  double s[3];
  for (int d = 0; d < 3; ++d) {
    if (M[d] < 1 || !(L[d] > 0)) return -1;
    s[d] = (double)M[d] / L[d];
  }
  for (int64_t i = 0; i < n; ++i) {
    const double p[3] = {x[i], y[i], z[i]};
    int32_t k[3];
    for (int d = 0; d < 3; ++d) {
      double f = floor(p[d] * s[d]);
      int32_t kk = (f < 0.0) ? 0 : (f > (double)(M[d] - 1) ? M[d] - 1 : (int32_t)f);
      k[d] = kk;
    }
    cell[i] = k[0] + M[0] * (k[1] + M[1] * k[2]);
  }
  return 0;
}

int ora_bin(int64_t n, const int32_t* cell, int64_t n_cells, int32_t* cnt, int32_t* cell_start,
            int32_t* cell_atoms) {
  if (n < 0 || n_cells < 1) return -1;
  for (int64_t c = 0; c < n_cells; ++c) cnt[c] = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (cell[i] < 0 || cell[i] >= n_cells) return -2;
    cnt[cell[i]]++;
  }
  cell_start[0] = 0;
  for (int64_t c = 0; c < n_cells; ++c) cell_start[c + 1] = cell_start[c] + cnt[c];
  /* stable placement: atoms visited in ascending index */
  int32_t* fill = (int32_t*)calloc((size_t)n_cells, sizeof(int32_t));
  if (!fill) return -3;
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = cell[i];
    cell_atoms[cell_start[c] + fill[c]] = (int32_t)i;
    fill[c]++;
  }
  free(fill);
  return 0;
}

/* ---------- Lennard-Jones, Eq. (2) ---------- */
static int excluded(int64_t i, int64_t j, int32_t chain_len, int32_t depth) {
  if (i / chain_len != j / chain_len) return 0;
  int64_t d = i > j ? i - j : j - i;
  return d <= depth;
}

/* pair parameters by Lorentz-Berthelot mixing */
static void lj_params(const ora_ff* ff, int ti, int tj, double* sig, double* eps) {
  *sig = 0.5 * (ff->sigma[ti] + ff->sigma[tj]);
  *eps = sqrt(ff->epsilon[ti] * ff->epsilon[tj]);
}

/* energy and the scalar g with F_i = g * (x_i - x_j), for r^2 < rc^2 */
static double lj_pair(double sig, double eps, double r2, double* g) {
  double s2 = sig * sig / r2;
  double s6 = s2 * s2 * s2;
  double s12 = s6 * s6;
  *g = 24.0 * eps * (2.0 * s12 - s6) / r2;
  return 4.0 * eps * (s12 - s6);
}

static double lj_energy_at(double sig, double eps, double r) {
  double s6 = pow(sig / r, 6.0);
  return 4.0 * eps * (s6 * s6 - s6);
}

int ora_lj_brute(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                 const double* z, const uint8_t* type, const double L[3], double* fx, double* fy,
                 double* fz, ora_energy* e) {
  if (!ff || n < 0 || chain_len < 1) return -1;
  const double rc2 = ff->rc * ff->rc;
  nsum E = {0, 0}, Es = {0, 0}, W = {0, 0};
  for (int64_t i = 0; i < n; ++i) fx[i] = fy[i] = fz[i] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      if (excluded(i, j, chain_len, ff->excl_depth)) continue;
      double dx = min_image(x[i] - x[j], L[0]);
      double dy = min_image(y[i] - y[j], L[1]);
      double dz = min_image(z[i] - z[j], L[2]);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < rc2)) continue;
      double sig, eps, g;
      lj_params(ff, type[i], type[j], &sig, &eps);
      double en = lj_pair(sig, eps, r2, &g);
      fx[i] += g * dx; fy[i] += g * dy; fz[i] += g * dz;
      fx[j] -= g * dx; fy[j] -= g * dy; fz[j] -= g * dz;
      nadd(&E, en);
      nadd(&Es, en - lj_energy_at(sig, eps, ff->rc));
      nadd(&W, g * r2);
    }
  }
  if (e) {
    e->e_lj = nval(&E);
    e->e_lj_shifted = nval(&Es);
    e->virial_lj = nval(&W);
  }
  return 0;
}

int ora_lj_cells(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                 const double* z, const uint8_t* type, const double L[3], const int32_t M[3],
                 int32_t R, const int64_t* subset, int64_t n_subset, double* fx, double* fy,
                 double* fz, ora_energy* e) {
  if (!ff || n < 0 || chain_len < 1 || R < 1) return -1;
  for (int d = 0; d < 3; ++d) {
    if (M[d] < 2 * R + 1) return -2;                            /* a cell would be visited twice */
    if (L[d] / M[d] * R < ff->rc) return -3;                    /* stencil would not reach rc */
  }
  const int64_t n_cells = (int64_t)M[0] * M[1] * M[2];
  int32_t* cell = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* cnt = (int32_t*)malloc((size_t)n_cells * sizeof(int32_t));
  int32_t* start = (int32_t*)malloc((size_t)(n_cells + 1) * sizeof(int32_t));
  int32_t* atoms = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  double* ei = NULL; double* esi = NULL; double* wi = NULL;
  if (!subset) {
    ei = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    esi = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    wi = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  }
  if (!cell || !cnt || !start || !atoms || (!subset && (!ei || !esi || !wi))) return -4;
  for (int64_t i = 0; i < n; ++i)   /* the grid search assumes wrapped coordinates */
    if (!(x[i] >= 0 && x[i] < L[0] && y[i] >= 0 && y[i] < L[1] && z[i] >= 0 && z[i] < L[2])) {
      free(cell); free(cnt); free(start); free(atoms); free(ei); free(esi); free(wi);
      return -6;
    }
  ora_cell_index(n, x, y, z, L, M, cell);
  ora_bin(n, cell, n_cells, cnt, start, atoms);
  const double rc2 = ff->rc * ff->rc;
  const int64_t n_home = subset ? n_subset : n;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
  for (int64_t h = 0; h < n_home; ++h) {
    const int64_t i = subset ? subset[h] : h;
    if (i < 0 || i >= n) { bad = 1; continue; }
    const int32_t c = cell[i];
    const int32_t kx = c % M[0], ky = (c / M[0]) % M[1], kz = c / (M[0] * M[1]);
    double ax = 0, ay = 0, az = 0;
    nsum E = {0, 0}, Es = {0, 0}, W = {0, 0};
    for (int32_t oz = -R; oz <= R; ++oz)
      for (int32_t oy = -R; oy <= R; ++oy)
        for (int32_t ox = -R; ox <= R; ++ox) {
          int32_t nx = (kx + ox + M[0]) % M[0];
          int32_t ny = (ky + oy + M[1]) % M[1];
          int32_t nz = (kz + oz + M[2]) % M[2];
          int32_t nc = nx + M[0] * (ny + M[1] * nz);
          for (int32_t s = start[nc]; s < start[nc + 1]; ++s) {
            int64_t j = atoms[s];
            if (j == i || excluded(i, j, chain_len, ff->excl_depth)) continue;
            double dx = min_image(x[i] - x[j], L[0]);
            double dy = min_image(y[i] - y[j], L[1]);
            double dz = min_image(z[i] - z[j], L[2]);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < rc2)) continue;
            double sig, eps, g;
            lj_params(ff, type[i], type[j], &sig, &eps);
            double en = lj_pair(sig, eps, r2, &g);
            ax += g * dx; ay += g * dy; az += g * dz;
            nadd(&E, 0.5 * en);
            nadd(&Es, 0.5 * (en - lj_energy_at(sig, eps, ff->rc)));
            nadd(&W, 0.5 * g * r2);
          }
        }
    fx[i] = ax; fy[i] = ay; fz[i] = az;
    if (!subset) { ei[i] = nval(&E); esi[i] = nval(&Es); wi[i] = nval(&W); }
  }
  if (e && !subset) {
    e->e_lj = ora_sum(n, ei);
    e->e_lj_shifted = ora_sum(n, esi);
    e->virial_lj = ora_sum(n, wi);
  }
  free(cell); free(cnt); free(start); free(atoms); free(ei); free(esi); free(wi);
  return bad ? -5 : 0;
}

/* ---------- bonded terms, Eqs. (4)-(6) ---------- */
static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* Eq. (4).  f[0..2] force on i, f[3..5] on j. */
double ora_bond_term(const ora_ff* ff, const double* xi, const double* xj, double* f) {
  double d[3];
  sub3(xj, xi, d);                    /* from i to j */
  double r = norm3(d);
  double dr = r - ff->b0;
  /* E = kb/2 (r-b)^2, dE/dx_i = -kb (r-b) d/r */
  double g = ff->kb * dr / r;
  for (int k = 0; k < 3; ++k) { f[k] = g * d[k]; f[3 + k] = -g * d[k]; }
  return 0.5 * ff->kb * dr * dr;
}

/* Eq. (5), theta = angle i-j-k at j.  f: 9 doubles (i, j, k). */
double ora_angle_term(const ora_ff* ff, const double* xi, const double* xj, const double* xk,
                      double* f, double* theta_out) {
  double a[3], c[3], ac[3];
  sub3(xi, xj, a);
  sub3(xk, xj, c);
  cross3(a, c, ac);
  double la = norm3(a), lc = norm3(c);
  double theta = atan2(norm3(ac), dot3(a, c));
  double th0 = ff->theta0_deg * M_PI / 180.0;
  double dth = theta - th0;
  double cth = cos(theta), sth = sin(theta);
  if (sth < 1e-12) sth = 1e-12;
  /* F_i = ka (theta - theta0) / sin(theta) * (c/(|a||c|) - cos(theta) a/|a|^2) */
  double gk = ff->ka * dth / sth;
  for (int k = 0; k < 3; ++k) {
    double fi = gk * (c[k] / (la * lc) - cth * a[k] / (la * la));
    double fk = gk * (a[k] / (la * lc) - cth * c[k] / (lc * lc));
    f[k] = fi;
    f[6 + k] = fk;
    f[3 + k] = -fi - fk;
  }
  if (theta_out) *theta_out = theta;
  return 0.5 * ff->ka * dth * dth;
}

/* Eq. (6), phi = dihedral i-j-k-l (IUPAC: trans = pi).  f: 12 doubles.
   Gradient of phi after Blondel & Karplus, J. Comput. Chem. 17 (1996) 1132. */
double ora_dihedral_term(const ora_ff* ff, const double* xi, const double* xj, const double* xk,
                         const double* xl, double* f, double* phi_out) {
  double F[3], G[3], H[3], A[3], B[3], BA[3];
  sub3(xi, xj, F);
  sub3(xj, xk, G);
  sub3(xl, xk, H);
  cross3(F, G, A);
  cross3(H, G, B);
  cross3(B, A, BA);
  double A2 = dot3(A, A), B2 = dot3(B, B), lG = norm3(G);
  double lA = sqrt(A2), lB = sqrt(B2);
  double cphi = dot3(A, B) / (lA * lB);
  double sphi = dot3(BA, G) / (lA * lB * lG);
  double phi = atan2(sphi, cphi);
  double n = (double)ff->n_dih;
  double phis = ff->phis_deg * M_PI / 180.0;
  double energy = ff->kphi * (1.0 + cos(n * phi - phis));
  double dEdphi = -n * ff->kphi * sin(n * phi - phis);
  double FG = dot3(F, G), HG = dot3(H, G);
  for (int k = 0; k < 3; ++k) {
    double dpi = -lG / A2 * A[k];
    double dpl = lG / B2 * B[k];
    double dpj = lG / A2 * A[k] + FG / (A2 * lG) * A[k] - HG / (B2 * lG) * B[k];
    double dpk = HG / (B2 * lG) * B[k] - FG / (A2 * lG) * A[k] - lG / B2 * B[k];
    f[k] = -dEdphi * dpi;
    f[3 + k] = -dEdphi * dpj;
    f[6 + k] = -dEdphi * dpk;
    f[9 + k] = -dEdphi * dpl;
  }
  if (phi_out) *phi_out = phi;
  return energy;
}

/* unwrapped copy of sites p..p+k-1 of a chain, relative to site p, minimum-imaged link by link */
static void local_sites(const double* x, const double* y, const double* z, const double L[3],
                        int64_t p, int k, double out[4][3]) {
  out[0][0] = x[p]; out[0][1] = y[p]; out[0][2] = z[p];
  for (int s = 1; s < k; ++s) {
    double d[3] = {x[p + s] - x[p + s - 1], y[p + s] - y[p + s - 1], z[p + s] - z[p + s - 1]};
    for (int q = 0; q < 3; ++q) out[s][q] = out[s - 1][q] + min_image(d[q], L[q]);
  }
}

/* A term of k consecutive sites (k = 2 bond, 3 angle, 4 dihedral) starting at site q
   of a linear chain exists iff it ends inside the chain. */
static int term_exists(int64_t q, int32_t k, int32_t chain_len) { return q + k - 1 < chain_len; }

int ora_chain_terms(int32_t chain_len, int32_t k, int32_t* out, int32_t max_terms) {
  if (chain_len < 1 || k < 2 || k > 4) return -1;
  int32_t m = 0;
  for (int32_t q = 0; q < chain_len; ++q) {
    if (!term_exists(q, k, chain_len)) continue;
    if (m < max_terms)
      for (int32_t a = 0; a < k; ++a) out[m * k + a] = q + a;
    ++m;
  }
  return m;
}

int ora_bonded(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
               const double* z, const double L[3], double* fx, double* fy, double* fz,
               ora_energy* e) {
  if (!ff || n < 0 || chain_len < 1 || n % chain_len) return -1;
  nsum Eb = {0, 0}, Ea = {0, 0}, Ed = {0, 0}, W = {0, 0};
  for (int64_t p = 0; p < n; ++p) {
    int64_t q = p % chain_len;           /* site index within its chain */
    double s[4][3], f[12];
    if (term_exists(q, 2, chain_len)) {
      local_sites(x, y, z, L, p, 2, s);
      nadd(&Eb, ora_bond_term(ff, s[0], s[1], f));
      for (int a = 0; a < 2; ++a) {
        fx[p + a] += f[3 * a]; fy[p + a] += f[3 * a + 1]; fz[p + a] += f[3 * a + 2];
      }
      double w = 0;
      for (int a = 1; a < 2; ++a)
        for (int k = 0; k < 3; ++k) w += (s[a][k] - s[0][k]) * f[3 * a + k];
      nadd(&W, w);
    }
    if (term_exists(q, 3, chain_len)) {
      local_sites(x, y, z, L, p, 3, s);
      nadd(&Ea, ora_angle_term(ff, s[0], s[1], s[2], f, NULL));
      for (int a = 0; a < 3; ++a) {
        fx[p + a] += f[3 * a]; fy[p + a] += f[3 * a + 1]; fz[p + a] += f[3 * a + 2];
      }
      double w = 0;
      for (int a = 1; a < 3; ++a)
        for (int k = 0; k < 3; ++k) w += (s[a][k] - s[0][k]) * f[3 * a + k];
      nadd(&W, w);
    }
    if (term_exists(q, 4, chain_len)) {
      local_sites(x, y, z, L, p, 4, s);
      nadd(&Ed, ora_dihedral_term(ff, s[0], s[1], s[2], s[3], f, NULL));
      for (int a = 0; a < 4; ++a) {
        fx[p + a] += f[3 * a]; fy[p + a] += f[3 * a + 1]; fz[p + a] += f[3 * a + 2];
      }
      double w = 0;
      for (int a = 1; a < 4; ++a)
        for (int k = 0; k < 3; ++k) w += (s[a][k] - s[0][k]) * f[3 * a + k];
      nadd(&W, w);
    }
  }
  if (e) {
    e->e_bond = nval(&Eb);
    e->e_angle = nval(&Ea);
    e->e_dih = nval(&Ed);
    e->virial_bonded = nval(&W);
  }
  return 0;
}

int ora_forces(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
               const double* z, const uint8_t* type, const double L[3], const int32_t M[3],
               int32_t R, double* fx, double* fy, double* fz, ora_energy* e) {
  ora_energy tmp;
  memset(&tmp, 0, sizeof tmp);
  int rc = ora_lj_cells(ff, n, chain_len, x, y, z, type, L, M, R, NULL, 0, fx, fy, fz, &tmp);
  if (rc) return rc;
  rc = ora_bonded(ff, n, chain_len, x, y, z, L, fx, fy, fz, &tmp);
  if (rc) return rc;
  if (e) *e = tmp;
  return 0;
}

int ora_kinetic(const ora_ff* ff, int64_t n, const double* vx, const double* vy, const double* vz,
                const uint8_t* type, double* ke, double* temperature) {
  if (!ff || n < 2) return -1;
  nsum K = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double m = ff->mass[type[i]];
    nadd(&K, 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) / ACC_UNIT);
  }
  double k = nval(&K);
  if (ke) *ke = k;
  if (temperature) *temperature = 2.0 * k / ((double)(3 * n - 3) * R_GAS);
  return 0;
}

int ora_com_velocity(const ora_ff* ff, int64_t n, const double* vx, const double* vy, const double* vz,
                     const uint8_t* type, double u[3]) {
  if (!ff || n < 1 || !u) return -1;
  nsum P[3] = {{0, 0}, {0, 0}, {0, 0}}, Mt = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double m = ff->mass[type[i]];
    nadd(&P[0], m * vx[i]);
    nadd(&P[1], m * vy[i]);
    nadd(&P[2], m * vz[i]);
    nadd(&Mt, m);
  }
  for (int d = 0; d < 3; ++d) u[d] = nval(&P[d]) / nval(&Mt);
  return 0;
}

static void remove_com_velocity(const ora_ff* ff, int64_t n, double* vx, double* vy, double* vz,
                                const uint8_t* type) {
  double u[3];
  ora_com_velocity(ff, n, vx, vy, vz, type, u);
  for (int64_t i = 0; i < n; ++i) {
    vx[i] -= u[0];
    vy[i] -= u[1];
    vz[i] -= u[2];
  }
}

int ora_run(const ora_ff* ff, const ora_integ* in, int64_t n, int32_t chain_len, double* x,
            double* y, double* z, double* vx, double* vy, double* vz, double* fx, double* fy,
            double* fz, const uint8_t* type, const double L[3], const int32_t M[3], int32_t R,
            int32_t n_steps, ora_energy* e_out, double* ke_out, double* t_out) {
  if (!ff || !in || n < 2 || n_steps < 0 || !(in->dt > 0)) return -1;
  const double h = 0.5 * in->dt;
  ora_energy e;
  memset(&e, 0, sizeof e);
  double ke = 0, T = 0;
  for (int32_t step = 0; step < n_steps; ++step) {
    for (int64_t i = 0; i < n; ++i) {
      double a = ACC_UNIT / ff->mass[type[i]];
      vx[i] += h * (a * fx[i]);
      vy[i] += h * (a * fy[i]);
      vz[i] += h * (a * fz[i]);
      x[i] += in->dt * vx[i];
      y[i] += in->dt * vy[i];
      z[i] += in->dt * vz[i];
    }
    ora_wrap(n, x, y, z, L);
    int rc = ora_forces(ff, n, chain_len, x, y, z, type, L, M, R, fx, fy, fz, &e);
    if (rc) return rc;
    for (int64_t i = 0; i < n; ++i) {
      double a = ACC_UNIT / ff->mass[type[i]];
      vx[i] += h * (a * fx[i]);
      vy[i] += h * (a * fy[i]);
      vz[i] += h * (a * fz[i]);
    }
    if (in->remove_com) remove_com_velocity(ff, n, vx, vy, vz, type);
    ora_kinetic(ff, n, vx, vy, vz, type, &ke, &T);
    if (in->T0 > 0 && T > 0) {
      double lam = sqrt(1.0 + in->dt / in->tau * (in->T0 / T - 1.0));
      for (int64_t i = 0; i < n; ++i) { vx[i] *= lam; vy[i] *= lam; vz[i] *= lam; }
    }
  }
  if (e_out) *e_out = e;
  if (ke_out) *ke_out = ke;
  if (t_out) *t_out = T;
  return 0;
}

int ora_run_leapfrog(const ora_ff* ff, const ora_integ* in, ora_nh* nh, int64_t n, int32_t chain_len,
                     double* x, double* y, double* z, double* vx, double* vy, double* vz, double* fx,
                     double* fy, double* fz, const uint8_t* type, const double L[3], const int32_t M[3],
                     int32_t R, int32_t n_steps, ora_energy* e_out, double* ke_out, double* t_out) {
  if (!ff || !in || n < 2 || n_steps < 0 || !(in->dt > 0) || !(in->tau > 0)) return -1;
  const double dt = in->dt;
  const double two_pi = 6.283185307179586;
  const double omega2 = (two_pi / in->tau) * (two_pi / in->tau);
  double xi = nh ? nh->xi : 0.0, eta = nh ? nh->eta : 0.0;
  ora_energy e;
  memset(&e, 0, sizeof e);
  double ke = 0, T = 0;
  for (int32_t step = 0; step < n_steps; ++step) {
    /* v(t + dt/2) from v(t - dt/2): the friction term -xi v is taken at the middle of
       the interval, (v(t - dt/2) + v(t + dt/2)) / 2, which gives the division below */
    const double num = 1.0 - 0.5 * dt * xi, den = 1.0 + 0.5 * dt * xi;
    for (int64_t i = 0; i < n; ++i) {
      double a = ACC_UNIT / ff->mass[type[i]];
      vx[i] = (num * vx[i] + dt * (a * fx[i])) / den;
      vy[i] = (num * vy[i] + dt * (a * fy[i])) / den;
      vz[i] = (num * vz[i] + dt * (a * fz[i])) / den;
      x[i] += dt * vx[i];
      y[i] += dt * vy[i];
      z[i] += dt * vz[i];
    }
    ora_wrap(n, x, y, z, L);
    int rc = ora_forces(ff, n, chain_len, x, y, z, type, L, M, R, fx, fy, fz, &e);
    if (rc) return rc;
    if (in->remove_com) remove_com_velocity(ff, n, vx, vy, vz, type);
    ora_kinetic(ff, n, vx, vy, vz, type, &ke, &T);
    if (in->T0 > 0) {
      /* dxi/dt = omega^2 (T/T0 - 1) with T at the half step between xi(t) and xi(t + dt) */
      const double xi_next = xi + dt * omega2 * (T / in->T0 - 1.0);
      eta += 0.5 * dt * (xi + xi_next);
      xi = xi_next;
    }
  }
  if (nh) {
    nh->xi = xi;
    nh->eta = eta;
    nh->e_thermostat = in->T0 > 0 ? (double)(3 * n - 3) * R_GAS * in->T0 * (xi * xi / (2.0 * omega2) + eta) : 0.0;
  }
  if (e_out) *e_out = e;
  if (ke_out) *ke_out = ke;
  if (t_out) *t_out = T;
  return 0;
}

/* ---------- Section 5 observables ---------- */

static int32_t distance_bin(double r2, double dr, int32_t n_bins) {
  /* the largest k with (k dr)^2 <= r2; r2 < (n_bins dr)^2 is checked by the caller */
  int32_t k = (int32_t)(sqrt(r2) / dr);
  if (k > n_bins - 1) k = n_bins - 1;
  while (k > 0 && r2 < (k * dr) * (k * dr)) --k;
  while (k + 1 < n_bins && r2 >= ((k + 1) * dr) * ((k + 1) * dr)) ++k;
  return k;
}

static double pair_r2(const double* x, const double* y, const double* z, const double L[3], int64_t i,
                      int64_t j) {
  double dx = min_image(x[i] - x[j], L[0]);
  double dy = min_image(y[i] - y[j], L[1]);
  double dz = min_image(z[i] - z[j], L[2]);
  return dx * dx + dy * dy + dz * dz;
}

int ora_pair_histogram(int64_t n, int32_t chain_len, int32_t excl_depth, const double* x, const double* y,
                       const double* z, const double L[3], const int32_t* M, double rmax, int32_t n_bins,
                       uint64_t* counts) {
  if (n < 0 || chain_len < 1 || excl_depth < 0 || n_bins < 1 || !(rmax > 0) || !counts) return -1;
  const double dr = rmax / n_bins, rmax2 = (n_bins * dr) * (n_bins * dr);
  memset(counts, 0, sizeof(uint64_t) * (size_t)n_bins);
  if (!M) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j) {
        if (excluded(i, j, chain_len, excl_depth)) continue;
        double r2 = pair_r2(x, y, z, L, i, j);
        if (r2 < rmax2) ++counts[distance_bin(r2, dr, n_bins)];
      }
    return 0;
  }
  for (int d = 0; d < 3; ++d)
    if (M[d] < 3 || L[d] / M[d] < rmax) return -2;
  const int64_t n_cells = (int64_t)M[0] * M[1] * M[2];
  int32_t* cell = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* cnt = (int32_t*)malloc((size_t)n_cells * sizeof(int32_t));
  int32_t* start = (int32_t*)malloc((size_t)(n_cells + 1) * sizeof(int32_t));
  int32_t* atoms = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!cell || !cnt || !start || !atoms) { free(cell); free(cnt); free(start); free(atoms); return -4; }
  ora_cell_index(n, x, y, z, L, M, cell);
  ora_bin(n, cell, n_cells, cnt, start, atoms);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = cell[i];
    const int32_t kx = c % M[0], ky = (c / M[0]) % M[1], kz = c / (M[0] * M[1]);
    for (int32_t oz = -1; oz <= 1; ++oz)
      for (int32_t oy = -1; oy <= 1; ++oy)
        for (int32_t ox = -1; ox <= 1; ++ox) {
          int32_t nc = (kx + ox + M[0]) % M[0] + M[0] * ((ky + oy + M[1]) % M[1] + M[1] * ((kz + oz + M[2]) % M[2]));
          for (int32_t s = start[nc]; s < start[nc + 1]; ++s) {
            int64_t j = atoms[s];
            if (j <= i || excluded(i, j, chain_len, excl_depth)) continue;
            double r2 = pair_r2(x, y, z, L, i, j);
            if (r2 < rmax2) ++counts[distance_bin(r2, dr, n_bins)];
          }
        }
  }
  free(cell); free(cnt); free(start); free(atoms);
  return 0;
}

int ora_dihedral_stats(int64_t n, int32_t chain_len, const double* x, const double* y, const double* z,
                       const double L[3], int32_t n_bins, uint64_t* hist, uint64_t classes[3]) {
  if (n < 0 || chain_len < 4 || n % chain_len || n_bins < 0 || (n_bins > 0 && !hist) || !classes) return -1;
  ora_ff ff;
  memset(&ff, 0, sizeof ff);
  ff.n_dih = 1;
  if (n_bins > 0) memset(hist, 0, sizeof(uint64_t) * (size_t)n_bins);
  classes[0] = classes[1] = classes[2] = 0;
  const double two_pi = 2.0 * M_PI, third = two_pi / 3.0, scale = n_bins / two_pi;
  for (int64_t p = 0; p < n; ++p) {
    if (!term_exists(p % chain_len, 4, chain_len)) continue;
    double s[4][3], f[12], phi;
    local_sites(x, y, z, L, p, 4, s);
    ora_dihedral_term(&ff, s[0], s[1], s[2], s[3], f, &phi);
    if (n_bins > 0) {
      int32_t k = (int32_t)floor((phi + M_PI) * scale);
      if (k > n_bins - 1) k = n_bins - 1;
      if (k < 0) k = 0;
      ++hist[k];
    }
    if (fabs(phi) > third) ++classes[0];
    else if (phi >= 0) ++classes[1];
    else ++classes[2];
  }
  return 0;
}

int ora_chain_shape(const ora_ff* ff, int64_t n, int32_t chain_len, const double* x, const double* y,
                    const double* z, const uint8_t* type, const double L[3], double* out) {
  if (!ff || n < 0 || chain_len < 1 || n % chain_len || !out) return -1;
  double* u = (double*)malloc(sizeof(double) * 3 * (size_t)chain_len);
  if (!u) return -4;
  for (int64_t c = 0; c < n / chain_len; ++c) {
    const int64_t a = c * chain_len;
    u[0] = x[a]; u[1] = y[a]; u[2] = z[a];
    for (int32_t p = 1; p < chain_len; ++p) {
      u[3 * p + 0] = u[3 * (p - 1) + 0] + min_image(x[a + p] - x[a + p - 1], L[0]);
      u[3 * p + 1] = u[3 * (p - 1) + 1] + min_image(y[a + p] - y[a + p - 1], L[1]);
      u[3 * p + 2] = u[3 * (p - 1) + 2] + min_image(z[a + p] - z[a + p - 1], L[2]);
    }
    double msum = 0, cm[3] = {0, 0, 0};
    for (int32_t p = 0; p < chain_len; ++p) {
      const double m = ff->mass[type[a + p]];
      msum += m;
      for (int q = 0; q < 3; ++q) cm[q] += m * u[3 * p + q];
    }
    for (int q = 0; q < 3; ++q) cm[q] /= msum;
    double rg = 0;
    for (int32_t p = 0; p < chain_len; ++p) {
      const double m = ff->mass[type[a + p]];
      double d2 = 0;
      for (int q = 0; q < 3; ++q) d2 += (u[3 * p + q] - cm[q]) * (u[3 * p + q] - cm[q]);
      rg += m * d2;
    }
    out[4 * c] = rg / msum;
    for (int q = 0; q < 3; ++q) out[4 * c + 1 + q] = u[3 * (chain_len - 1) + q] - u[q];
  }
  free(u);
  return 0;
}

/* The end-to-end vector of the chain starting at atom a: its bonds, minimum-imaged, summed
   from the first to the last. */
static void end_to_end(int64_t a, int32_t chain_len, const double* x, const double* y, const double* z,
                       const double L[3], double r[3]) {
  r[0] = r[1] = r[2] = 0.0;
  for (int32_t p = 1; p < chain_len; ++p) {
    r[0] += min_image(x[a + p] - x[a + p - 1], L[0]);
    r[1] += min_image(y[a + p] - y[a + p - 1], L[1]);
    r[2] += min_image(z[a + p] - z[a + p - 1], L[2]);
  }
}

int ora_ree_acf(int64_t n, int32_t chain_len, const double* x0, const double* y0, const double* z0,
                const double* x, const double* y, const double* z, const double L[3], double* acf) {
  if (n <= 0 || chain_len < 2 || n % chain_len || !acf) return -1;
  nsum num = {0, 0}, den = {0, 0};
  for (int64_t a = 0; a < n; a += chain_len) {
    double r0[3], r[3];
    end_to_end(a, chain_len, x0, y0, z0, L, r0);
    end_to_end(a, chain_len, x, y, z, L, r);
    nadd(&num, dot3(r, r0));
    nadd(&den, dot3(r0, r0));
  }
  *acf = nval(&num) / nval(&den);
  return 0;
}
