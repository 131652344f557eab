/* Seeded self-avoiding growth of united-atom polyethylene chains in a periodic cube.
 *
 * Input generation only: nothing here is part of the simulated method.  The melt
 * recipe (bond 1.53 A, angle 109.47 deg, dihedral 180 / +60 / -60 deg with
 * probabilities 0.6 / 0.2 / 0.2, clearance d_min from every placed atom except the
 * same chain's three predecessors, up to n_draws draws per site) follows the
 * united-atom chain model of the paper's Section 2.  Chains grow in lock-step (atom p
 * of every chain before atom p+1 of any), so crowding is spread over the whole box.
 * When no draw at a site is clear, the chain's last few atoms are regrown with fresh
 * draws (depth 1..max_depth, bounded attempts); if that also fails, the old atoms are
 * restored and the site's torsion is drawn freely in [0, 2pi) (the rotational states
 * put every chain on a diamond lattice, where a self-trapped walk has no clear
 * state); the first clear free draw, else the clearest draw of all, is taken.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), 53-bit uniforms, Box-Muller normals.
 * Build: gcc -O2 -shared -fPIC grow.c -o libgrow.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } rng_t;

static uint64_t sm64(rng_t* r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static double uni(rng_t* r) { return (double)(sm64(r) >> 11) * (1.0 / 9007199254740992.0); }
static double gauss(rng_t* r) {
  double u1 = 1.0 - uni(r);            /* (0, 1] */
  double u2 = uni(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

typedef struct {
  int G;            /* cells per dimension */
  double h, L;
  int32_t* head;    /* [G^3] first atom in cell, -1 empty */
  int32_t* next;    /* [N] */
  int32_t* cellof;  /* [N] */
  double* w;        /* [N*3] wrapped positions */
} grid_t;

static double wrap1(double x, double L) {
  double y = x - L * floor(x / L);
  if (y >= L) y -= L;
  if (y < 0) y += L;
  return y;
}

static int cell_of(const grid_t* g, const double* w) {
  int c[3];
  for (int d = 0; d < 3; ++d) {
    int k = (int)floor(w[d] / g->h);
    if (k < 0) k = 0;
    if (k >= g->G) k = g->G - 1;
    c[d] = k;
  }
  return (c[0] * g->G + c[1]) * g->G + c[2];
}

static void grid_insert(grid_t* g, int id, const double* p) {
  double* w = g->w + 3 * (size_t)id;
  for (int d = 0; d < 3; ++d) w[d] = wrap1(p[d], g->L);
  int c = cell_of(g, w);
  g->cellof[id] = c;
  g->next[id] = g->head[c];
  g->head[c] = id;
}

static void grid_remove(grid_t* g, int id) {
  int c = g->cellof[id];
  int32_t* pp = &g->head[c];
  while (*pp != -1) {
    if (*pp == id) { *pp = g->next[id]; break; }
    pp = &g->next[*pp];
  }
  g->cellof[id] = -1;
}

/* clearance of point p (unwrapped) for atom (chain, idx) */
static double clearance(const grid_t* g, const double* p, int chain, int idx, int chain_len) {
  double w[3];
  for (int d = 0; d < 3; ++d) w[d] = wrap1(p[d], g->L);
  int c0 = (int)floor(w[0] / g->h), c1 = (int)floor(w[1] / g->h), c2 = (int)floor(w[2] / g->h);
  if (c0 >= g->G) c0 = g->G - 1;
  if (c1 >= g->G) c1 = g->G - 1;
  if (c2 >= g->G) c2 = g->G - 1;
  double best2 = INFINITY;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int e = -1; e <= 1; ++e) {
        int x = (c0 + a + g->G) % g->G, y = (c1 + b + g->G) % g->G, z = (c2 + e + g->G) % g->G;
        for (int id = g->head[(x * g->G + y) * g->G + z]; id != -1; id = g->next[id]) {
          int oc = id / chain_len, oi = id % chain_len;
          if (oc == chain && abs(oi - idx) <= 3) continue;
          double r2 = 0;
          for (int d = 0; d < 3; ++d) {
            double dd = g->w[3 * (size_t)id + d] - w[d];
            dd -= g->L * nearbyint(dd / g->L);
            r2 += dd * dd;
          }
          if (r2 < best2) best2 = r2;
        }
      }
  return sqrt(best2);
}

static void unit3(double* v) {
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= n; v[1] /= n; v[2] /= n;
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

typedef struct {
  int n_chains, chain_len, n_draws;
  double L, bond, theta, d_min;
  double phi[3], pcum[3];
  double* P;   /* [N*3] unwrapped */
  grid_t g;
  rng_t rng;
} grower_t;

/* one random candidate for atom p of chain c; free_torsion draws the dihedral
   uniformly in [0, 2pi) instead of from the three rotational states */
static void candidate(grower_t* s, int c, int p, double* out, int free_torsion) {
  const double* base = s->P + 3 * (size_t)c * s->chain_len;
  if (p == 0) {
    for (int d = 0; d < 3; ++d) out[d] = uni(&s->rng) * s->L;
  } else if (p == 1) {
    double u[3] = {gauss(&s->rng), gauss(&s->rng), gauss(&s->rng)};
    unit3(u);
    for (int d = 0; d < 3; ++d) out[d] = base[d] + s->bond * u[d];
  } else if (p == 2) {
    const double* a = base;
    const double* b = base + 3;
    double ub[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    unit3(ub);
    double w[3] = {gauss(&s->rng), gauss(&s->rng), gauss(&s->rng)};
    double dot = w[0] * ub[0] + w[1] * ub[1] + w[2] * ub[2];
    for (int d = 0; d < 3; ++d) w[d] -= dot * ub[d];
    unit3(w);
    for (int d = 0; d < 3; ++d)
      out[d] = b[d] + s->bond * (-cos(s->theta) * ub[d] + sin(s->theta) * w[d]);
  } else {
    double u = uni(&s->rng);
    int k = u < s->pcum[0] ? 0 : (u < s->pcum[1] ? 1 : 2);
    double phi = free_torsion ? 6.283185307179586 * uni(&s->rng) : s->phi[k];
    const double* A = base + 3 * (p - 3);
    const double* B = base + 3 * (p - 2);
    const double* C = base + 3 * (p - 1);
    double bc[3] = {C[0] - B[0], C[1] - B[1], C[2] - B[2]};
    unit3(bc);
    double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double n[3];
    cross3(ab, bc, n);
    unit3(n);
    double m[3];
    cross3(n, bc, m);
    double x = -s->bond * cos(s->theta);
    double y = s->bond * sin(s->theta) * cos(phi);
    double z = s->bond * sin(s->theta) * sin(phi);
    for (int d = 0; d < 3; ++d) out[d] = C[d] + bc[d] * x + m[d] * y + n[d] * z;
  }
}

/* draw up to n_draws candidates; store the first clear one (return 1) or the best (return 0) */
static int try_site(grower_t* s, int c, int p, double* out, double* clr_out, int free_torsion) {
  double best = -1.0, cand[3];
  for (int t = 0; t < s->n_draws; ++t) {
    candidate(s, c, p, cand, free_torsion);
    double clr = clearance(&s->g, cand, c, p, s->chain_len);
    if (clr >= s->d_min) {
      memcpy(out, cand, sizeof cand);
      *clr_out = clr;
      return 1;
    }
    if (clr > best) { best = clr; memcpy(out, cand, sizeof cand); }
  }
  *clr_out = best;
  return 0;
}

static void set_atom(grower_t* s, int c, int p, const double* x) {
  int id = c * s->chain_len + p;
  memcpy(s->P + 3 * (size_t)id, x, 3 * sizeof(double));
  grid_insert(&s->g, id, x);
}

/* stats: [0] placements below d_min, [1] successful backtracks, [2] min clearance * 1e6 */
int pe_grow_melt(int n_chains, int chain_len, double L, uint64_t seed, double d_min, int n_draws,
                 int max_depth, int max_attempts, double* out_pos, int64_t* stats) {
  if (n_chains <= 0 || chain_len < 4 || L <= 0 || n_draws <= 0) return -1;
  grower_t s;
  memset(&s, 0, sizeof s);
  s.n_chains = n_chains; s.chain_len = chain_len; s.n_draws = n_draws;
  s.L = L; s.bond = 1.53; s.theta = 109.47 * M_PI / 180.0; s.d_min = d_min;
  s.phi[0] = M_PI; s.phi[1] = M_PI / 3.0; s.phi[2] = -M_PI / 3.0;
  s.pcum[0] = 0.6; s.pcum[1] = 0.8; s.pcum[2] = 1.0;
  s.P = out_pos;
  s.rng.s = seed;
  size_t N = (size_t)n_chains * chain_len;
  double cmin = d_min > 1.0 ? d_min : 1.0;
  s.g.G = (int)floor(L / cmin);
  if (s.g.G < 3) s.g.G = 3;
  s.g.h = L / s.g.G;
  s.g.L = L;
  size_t ncell = (size_t)s.g.G * s.g.G * s.g.G;
  s.g.head = (int32_t*)malloc(ncell * sizeof(int32_t));
  s.g.next = (int32_t*)malloc(N * sizeof(int32_t));
  s.g.cellof = (int32_t*)malloc(N * sizeof(int32_t));
  s.g.w = (double*)malloc(N * 3 * sizeof(double));
  if (!s.g.head || !s.g.next || !s.g.cellof || !s.g.w) return -2;
  for (size_t i = 0; i < ncell; ++i) s.g.head[i] = -1;
  for (size_t i = 0; i < N; ++i) s.g.cellof[i] = -1;
  int64_t forced = 0, backtracks = 0;
  double minclr = INFINITY;
  double keep[8][3];
  for (int p = 0; p < chain_len; ++p) {
    for (int c = 0; c < n_chains; ++c) {
      double x[3], clr;
      if (try_site(&s, c, p, x, &clr, 0)) {
        set_atom(&s, c, p, x);
        if (clr < minclr) minclr = clr;
        continue;
      }
      double best_x[3] = {x[0], x[1], x[2]}, best_clr = clr;
      int done = 0;
      /* per clearance tier (d_min, 0.9 d_min, 0.8 d_min): pass 0 regrows with
         rotational states, pass 1 frees the site torsion, pass 2 regrows with free
         torsions */
      for (int pass = 0; pass < 9 && !done; ++pass) {
        s.d_min = d_min * (pass < 3 ? 1.0 : (pass < 6 ? 0.9 : 0.8));
        if (pass % 3 == 1) {
          double y[3], cy;
          if (p >= 3 && try_site(&s, c, p, y, &cy, 1)) {
            set_atom(&s, c, p, y);
            if (cy < minclr) minclr = cy;
            if (cy < d_min) ++forced;
            done = 1;
          } else if (p >= 3 && cy > best_clr) {
            memcpy(best_x, y, sizeof y);
            best_clr = cy;
          }
          continue;
        }
        int free_t = pass % 3 == 2;
        for (int att = 0; att < max_attempts && !done && p >= 4; ++att) {
          int depth = 1 + att % max_depth;
          if (depth > p - 3) depth = p - 3;
          if (depth > 8) depth = 8;
          for (int k = 0; k < depth; ++k) {
            int q = p - depth + k;
            memcpy(keep[k], s.P + 3 * ((size_t)c * chain_len + q), 3 * sizeof(double));
            grid_remove(&s.g, c * chain_len + q);
          }
          int ok = 1;
          for (int k = 0; k < depth && ok; ++k) {
            double y[3], cy;
            int q = p - depth + k;
            ok = try_site(&s, c, q, y, &cy, free_t);
            if (ok) set_atom(&s, c, q, y);
          }
          double cp = 0;
          if (ok) ok = try_site(&s, c, p, x, &cp, free_t);
          if (ok) {
            set_atom(&s, c, p, x);
            if (cp < minclr) minclr = cp;
            if (cp < d_min) ++forced;
            ++backtracks;
            done = 1;
          } else {
            for (int k = 0; k < depth; ++k) {
              int id = c * chain_len + (p - depth + k);
              if (s.g.cellof[id] != -1) grid_remove(&s.g, id);
            }
            for (int k = 0; k < depth; ++k) set_atom(&s, c, p - depth + k, keep[k]);
          }
        }
      }
      s.d_min = d_min;
      if (!done) {
        set_atom(&s, c, p, best_x);
        if (best_clr < minclr) minclr = best_clr;
        ++forced;
      }
    }
  }
  free(s.g.head); free(s.g.next); free(s.g.cellof); free(s.g.w);
  if (stats) {
    stats[0] = forced;
    stats[1] = backtracks;
    stats[2] = (int64_t)(minclr * 1e6);
  }
  return 0;
}
