/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU, FP64 reference for the shift-free fast multipole method of
 * Kajima, "Summation of certain locally bilinear forms and its applications to the
 * Fast Multipole Method" (arXiv:2009.00767).  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library; the product
 * path (the HIP library) never does, and the two share no code.
 *
 * What is computed (all in FP64, plain loops, no blocking or fusion):
 *   - the exact quantity being approximated: the direct pair sum
 *     phi_i = sum_{j != i, r_ij > 0} q_j G(x_i, x_j),  E_i = -grad_i phi_i,
 *     G = log r in 2D and 1/r in 3D (Introduction; Appendix A.2.2 names the
 *     Coulomb pair potential);
 *   - the uniform tree of Section 2.1 items 1-5 (box of side S, 2^D children per
 *     box, levels 0..L, interaction lists from level 2 on);
 *   - the shift-free passes of Section 2.2.1: box vectors formed directly from the
 *     particles at every level (U-bar-1/U-bar-2 with a level-independent particle
 *     map, see the Note closing Section 2.2.2), the bilinear forms summed over
 *     the interaction list at every level (D-bar-1), evaluation of every level's
 *     linear form at the particle and summation over levels (D-bar-2 and
 *     F(v) = L_{m^l}(v)), plus the direct near field (E-2 of Section 2.1).
 *     The vector space V is realised as box-size-scaled truncated expansions:
 *     complex Laurent/Taylor coefficients of order p in 2D (Greengard 1988, the
 *     paper's ref. [101]) and solid harmonics of degree <= p in 3D;
 *   - the classical method of Section 2.1 (U-1, U-2 shift, D-1, D-2 shift, E-1,
 *     E-2) with the same tree, lists and order, used only as a cross-check; *   - in 2D, an adaptive depth for clustered inputs (a particle's tree stops at
 *     the first level whose 3 x 3 boxes around it hold at most near_max
 *     particles): each particle runs the shift-free method of its own depth;
 *   - the paper's own realisation of V in 3D (Appendix, STEP1-STEP5): n x n x n
 *     fixed point charges per box (the paper's 4 x 4 x 4 at offsets {-2, -1, 1,
 *     2} s / 5, or any other node set, e.g. Chebyshev points, Discussion (1)),
 *     Lagrange weights for the particle map, and the pair sum of point charges
 *     as the bilinear form; both box-local per level and in the root frame of
 *     STEP4-STEP5 with the child sums of U-bar-2 and the parent-to-child
 *     additions of D-bar-2.
 *   - the same point-charge realisation in 2D with the log kernel (n x n
 *     points per square box, the paper's 4 x 4 of Appendix STEP1 and Fig. 3),
 *     box-local per level.
 *
 * Conventions: a box at level k has side s_k = S / 2^k; the leaf coordinate of a
 * particle along axis d is min(floor((x_d - o_d) * (2^L / S)), 2^L - 1) evaluated
 * in FP64 exactly as written (no contraction).  Positions outside [o, o + S] or
 * NaN make every entry point return -2.  Box arrays are row-major with x fastest:
 * 2D box (ix, iy) -> iy * n + ix, 3D (ix, iy, iz) -> (iz * n + iy) * n + ix.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDOMAIN (-2)
#define ORC_ENOMEM (-3)

/* ------------------------------------------------------------------------- */
/* Neumaier's compensated summation (used by the direct sum only).           */
/* ------------------------------------------------------------------------- */
typedef struct {
  double s, c;
} nsum;

static void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------- */
/* Direct sum (the definition the FMM approximates).                          */
/* ------------------------------------------------------------------------- */
int oracle_direct(int dim, int64_t n, const double* pos, const double* q, int64_t nt,
                  const int64_t* tgt, double* pot, double* field) {
  if ((dim != 2 && dim != 3) || n < 0 || nt < 0) return ORC_EINVAL;
  if (!tgt) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nt; ++t) {
    int64_t i = tgt ? tgt[t] : t;
    nsum ph = {0, 0}, ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = pos[dim * i] - pos[dim * j];
      double dy = pos[dim * i + 1] - pos[dim * j + 1];
      double dz = dim == 3 ? pos[dim * i + 2] - pos[dim * j + 2] : 0.0;
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) continue;
      if (dim == 2) {
        /* G = log r ;  -grad_i G = -(x_i - x_j) / r^2 */
        nadd(&ph, q[j] * 0.5 * log(r2));
        nadd(&ex, -q[j] * dx / r2);
        nadd(&ey, -q[j] * dy / r2);
      } else {
        /* G = 1/r ;  -grad_i G = (x_i - x_j) / r^3 */
        double r = sqrt(r2);
        nadd(&ph, q[j] / r);
        double w = q[j] / (r2 * r);
        nadd(&ex, w * dx);
        nadd(&ey, w * dy);
        nadd(&ez, w * dz);
      }
    }
    pot[t] = nval(&ph);
    if (field) {
      field[dim * t] = nval(&ex);
      field[dim * t + 1] = nval(&ey);
      if (dim == 3) field[dim * t + 2] = nval(&ez);
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Tree (Section 2.1, items 1-5).                                            */
/* ------------------------------------------------------------------------- */
int64_t oracle_leaf_coord(double x, double origin, double side, int L) {
  int64_t nl = (int64_t)1 << L;
  double t = floor((x - origin) * ((double)nl / side));
  int64_t i = (int64_t)t;
  if (i > nl - 1) i = nl - 1;
  return i;
}

static int check_domain(int dim, int64_t n, const double* pos, const double* origin,
                        double side) {
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) {
      double x = pos[dim * i + d];
      if (!(x >= origin[d] && x <= origin[d] + side)) return ORC_EDOMAIN;
    }
  return ORC_OK;
}

/* Particles bucketed by leaf (row-major leaf id), in input order within a leaf. */
typedef struct {
  int dim, L;
  int64_t nl;      /* leaves per side */
  int64_t nleaf;   /* nl^dim */
  int64_t* lc;     /* [n * dim] leaf coordinates */
  int64_t* start;  /* [nleaf + 1] */
  int64_t* idx;    /* [n] particle ids grouped by leaf */
} tree;

static void tree_free(tree* t) {
  free(t->lc);
  free(t->start);
  free(t->idx);
}

static int64_t leaf_id(const tree* t, const int64_t* c) {
  if (t->dim == 2) return c[1] * t->nl + c[0];
  return (c[2] * t->nl + c[1]) * t->nl + c[0];
}

static int tree_build(tree* t, int dim, int64_t n, const double* pos, const double* origin,
                      double side, int L) {
  t->dim = dim;
  t->L = L;
  t->nl = (int64_t)1 << L;
  t->nleaf = dim == 2 ? t->nl * t->nl : t->nl * t->nl * t->nl;
  t->lc = malloc(sizeof(int64_t) * (size_t)(n * dim + 1));
  t->start = calloc((size_t)t->nleaf + 1, sizeof(int64_t));
  t->idx = malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!t->lc || !t->start || !t->idx) {
    tree_free(t);
    return ORC_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d)
      t->lc[dim * i + d] = oracle_leaf_coord(pos[dim * i + d], origin[d], side, L);
  for (int64_t i = 0; i < n; ++i) t->start[leaf_id(t, &t->lc[dim * i]) + 1]++;
  for (int64_t b = 0; b < t->nleaf; ++b) t->start[b + 1] += t->start[b];
  int64_t* fill = malloc(sizeof(int64_t) * (size_t)(t->nleaf + 1));
  if (!fill) {
    tree_free(t);
    return ORC_ENOMEM;
  }
  memcpy(fill, t->start, sizeof(int64_t) * (size_t)t->nleaf);
  for (int64_t i = 0; i < n; ++i) t->idx[fill[leaf_id(t, &t->lc[dim * i])]++] = i;
  free(fill);
  return ORC_OK;
}

/* Interaction list of box (tx, ty) at level k >= 2: children of the parent's
 * neighbours (parent included) that are not adjacent to the box itself.  Two
 * same-level boxes are adjacent when every index differs by at most one; the
 * domain is not periodic.  Returns the count, writes (bx, by) pairs. */
int oracle_ilist2d(int k, int64_t tx, int64_t ty, int64_t* out) {
  if (k < 2) return 0;
  int64_t nb = (int64_t)1 << k, np = nb >> 1, px = tx >> 1, py = ty >> 1;
  int cnt = 0;
  for (int64_t ny = py - 1; ny <= py + 1; ++ny)
    for (int64_t nx = px - 1; nx <= px + 1; ++nx) {
      if (nx < 0 || ny < 0 || nx >= np || ny >= np) continue;
      for (int64_t by = 2 * ny; by <= 2 * ny + 1; ++by)
        for (int64_t bx = 2 * nx; bx <= 2 * nx + 1; ++bx) {
          if (llabs(bx - tx) <= 1 && llabs(by - ty) <= 1) continue;
          out[2 * cnt] = bx;
          out[2 * cnt + 1] = by;
          ++cnt;
        }
    }
  return cnt;
}

int oracle_ilist3d(int k, int64_t tx, int64_t ty, int64_t tz, int64_t* out) {
  if (k < 2) return 0;
  int64_t nb = (int64_t)1 << k, np = nb >> 1, px = tx >> 1, py = ty >> 1, pz = tz >> 1;
  int cnt = 0;
  for (int64_t nz = pz - 1; nz <= pz + 1; ++nz)
    for (int64_t ny = py - 1; ny <= py + 1; ++ny)
      for (int64_t nx = px - 1; nx <= px + 1; ++nx) {
        if (nx < 0 || ny < 0 || nz < 0 || nx >= np || ny >= np || nz >= np) continue;
        for (int64_t bz = 2 * nz; bz <= 2 * nz + 1; ++bz)
          for (int64_t by = 2 * ny; by <= 2 * ny + 1; ++by)
            for (int64_t bx = 2 * nx; bx <= 2 * nx + 1; ++bx) {
              if (llabs(bx - tx) <= 1 && llabs(by - ty) <= 1 && llabs(bz - tz) <= 1) continue;
              out[3 * cnt] = bx;
              out[3 * cnt + 1] = by;
              out[3 * cnt + 2] = bz;
              ++cnt;
            }
      }
  return cnt;
}

/* ------------------------------------------------------------------------- */
/* Near field (E-2 of Section 2.1): direct sum over the particle's own leaf   */
/* and the adjacent leaves, j != i, r > 0.  Plain (uncompensated) sums.       */
/* ------------------------------------------------------------------------- */
static void near_field(const tree* t, const double* pos, const double* q, int64_t i,
                       double* phi, double* e) {
  int dim = t->dim;
  const int64_t* c = &t->lc[dim * i];
  double ph = 0, ex = 0, ey = 0, ez = 0;
  int64_t zlo = dim == 3 ? c[2] - 1 : 0, zhi = dim == 3 ? c[2] + 1 : 0;
  for (int64_t nz = zlo; nz <= zhi; ++nz)
    for (int64_t ny = c[1] - 1; ny <= c[1] + 1; ++ny)
      for (int64_t nx = c[0] - 1; nx <= c[0] + 1; ++nx) {
        if (nx < 0 || ny < 0 || nz < 0 || nx >= t->nl || ny >= t->nl || nz >= t->nl) continue;
        int64_t nc[3] = {nx, ny, nz};
        int64_t lf = leaf_id(t, nc);
        for (int64_t s = t->start[lf]; s < t->start[lf + 1]; ++s) {
          int64_t j = t->idx[s];
          if (j == i) continue;
          double dx = pos[dim * i] - pos[dim * j];
          double dy = pos[dim * i + 1] - pos[dim * j + 1];
          double dz = dim == 3 ? pos[dim * i + 2] - pos[dim * j + 2] : 0.0;
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0.0) continue;
          if (dim == 2) {
            ph += q[j] * 0.5 * log(r2);
            ex -= q[j] * dx / r2;
            ey -= q[j] * dy / r2;
          } else {
            double r = sqrt(r2);
            ph += q[j] / r;
            double w = q[j] / (r2 * r);
            ex += w * dx;
            ey += w * dy;
            ez += w * dz;
          }
        }
      }
  *phi = ph;
  e[0] = ex;
  e[1] = ey;
  if (dim == 3) e[2] = ez;
}

/* ========================================================================= */
/* 2D: complex Laurent / Taylor expansions of order p, scaled by box side.    */
/*                                                                           */
/* Box b at level k, centre z_b, side s.  For a charge q at z, w = (z - z_b)/s.*/
/*   moments : A_0 = sum q,   A_m = -(1/m) sum q w^m          (m = 1..p)      */
/*   far potential of the box at z: Re[ A_0 log(z - z_b)                       */
/*                                     + sum_m A_m (s / (z - z_b))^m ]         */
/*   locals  : potential near target centre z_t: Re sum_l B_l ((z - z_t)/s)^l  */
/*   M2L (Greengard's multipole-to-local lemma with z_0 = z_b - z_t = s u):    */
/*     B_0 += A_0 (log(-u) + log s) + sum_m A_m (-1)^m u^-m                    */
/*     B_l += -A_0 / (l u^l) + u^-l sum_m A_m (-1)^m C(l+m-1, m-1) u^-m        */
/* ========================================================================= */

static double binom(int n, int r) {
  if (r < 0 || r > n) return 0.0;
  double c = 1.0;
  for (int i = 1; i <= r; ++i) c = c * (double)(n - r + i) / (double)i;
  return c;
}

static cplx box_centre2d(const double* o, double s, int64_t ix, int64_t iy) {
  return CMPLX(o[0] + s * ((double)ix + 0.5), o[1] + s * ((double)iy + 0.5));
}

/* Moments of every box at level k, formed directly from the particles (no shift). */
static void p2m2d_level(const tree* t, const double* pos, const double* q, int k, int p,
                        double side, const double* o, cplx* A) {
  int64_t nb = (int64_t)1 << k, span = (int64_t)1 << (t->L - k);
  double s = side / (double)nb;
  int P = p + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < nb * nb; ++b) {
    int64_t bx = b % nb, by = b / nb;
    cplx zb = box_centre2d(o, s, bx, by);
    cplx* a = &A[b * P];
    for (int m = 0; m < P; ++m) a[m] = 0;
    for (int64_t ly = by * span; ly < (by + 1) * span; ++ly)
      for (int64_t lx = bx * span; lx < (bx + 1) * span; ++lx) {
        int64_t lf = ly * t->nl + lx;
        for (int64_t e = t->start[lf]; e < t->start[lf + 1]; ++e) {
          int64_t c = t->idx[e];
          cplx w = (CMPLX(pos[2 * c], pos[2 * c + 1]) - zb) / s;
          a[0] += q[c];
          cplx wm = 1.0;
          for (int m = 1; m <= p; ++m) {
            wm *= w;
            a[m] += -q[c] * wm / (double)m;
          }
        }
      }
  }
}

/* One multipole-to-local conversion: source coefficients a (about a centre at
 * offset u box sides from the target centre) added into target locals bl. */
static void m2l2d_one(int p, double s, cplx u, const cplx* a, cplx* bl) {
  cplx up[64]; /* up[m] = u^-m, m <= 2p */
  up[0] = 1.0;
  cplx ui = 1.0 / u;
  for (int m = 1; m <= 2 * p; ++m) up[m] = up[m - 1] * ui;
  cplx acc = a[0] * (clog(-u) + log(s));
  for (int m = 1; m <= p; ++m) acc += a[m] * (m % 2 ? -1.0 : 1.0) * up[m];
  bl[0] += acc;
  for (int l = 1; l <= p; ++l) {
    cplx sum = 0;
    for (int m = 1; m <= p; ++m)
      sum += a[m] * (m % 2 ? -1.0 : 1.0) * binom(l + m - 1, m - 1) * up[m];
    bl[l] += -a[0] * up[l] / (double)l + up[l] * sum;
  }
}

/* Locals of the marked target boxes at level k: sum over the interaction list. */
static void m2l2d_level(int k, int p, double side, const cplx* A, const char* want, cplx* B) {
  int64_t nb = (int64_t)1 << k;
  double s = side / (double)nb;
  int P = p + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < nb * nb; ++t) {
    cplx* bl = &B[t * P];
    for (int l = 0; l < P; ++l) bl[l] = 0;
    if (want && !want[t]) continue;
    int64_t tx = t % nb, ty = t / nb, il[2 * 27];
    int n = oracle_ilist2d(k, tx, ty, il);
    for (int i = 0; i < n; ++i) {
      cplx u = CMPLX((double)(il[2 * i] - tx), (double)(il[2 * i + 1] - ty));
      m2l2d_one(p, s, u, &A[(il[2 * i + 1] * nb + il[2 * i]) * P], bl);
    }
  }
}

/* Evaluate a local expansion b (about centre z_t, side s) at z: potential and
 * field -grad phi = (-Re g', +Im g') with g(z) = sum_l b_l ((z - z_t)/s)^l. */
static void l2p2d_one(int p, double s, cplx zt, const cplx* b, double x, double y,
                      double* phi, double* e) {
  cplx w = (CMPLX(x, y) - zt) / s;
  cplx g = 0, gp = 0, wl = 1.0;
  for (int l = 0; l <= p; ++l) {
    g += b[l] * wl;
    if (l < p) gp += (double)(l + 1) * b[l + 1] * wl;
    wl *= w;
  }
  gp /= s;
  *phi += creal(g);
  e[0] += -creal(gp);
  e[1] += cimag(gp);
}

/* Classical shifts (Section 2.1, U-2 and D-2), unscaled textbook forms. */
/* Multipole of a child (scaled with side sc, centre zc) re-expanded about the
 * parent centre zp (side sp), added into ap. */
static void m2m2d_one(int p, double sc, cplx zc, double sp, cplx zp, const cplx* ac, cplx* ap) {
  cplx a[64], z0 = zc - zp;
  a[0] = ac[0];
  for (int m = 1; m <= p; ++m) a[m] = ac[m] * pow(sc, m);
  ap[0] += a[0];
  for (int l = 1; l <= p; ++l) {
    cplx bsum = -a[0] * cpow(z0, l) / (double)l;
    for (int m = 1; m <= l; ++m) bsum += a[m] * cpow(z0, l - m) * binom(l - 1, m - 1);
    ap[l] += bsum / pow(sp, l);
  }
}

/* Local about the parent centre zp (scaled with sp) re-expanded about a child
 * centre zc (side sc), added into bc. */
static void l2l2d_one(int p, double sp, cplx zp, double sc, cplx zc, const cplx* bp, cplx* bc) {
  cplx c[64], d = zc - zp;
  for (int l = 0; l <= p; ++l) c[l] = bp[l] / pow(sp, l);
  for (int l = 0; l <= p; ++l) {
    cplx sum = 0;
    for (int m = l; m <= p; ++m) sum += c[m] * binom(m, l) * cpow(d, m - l);
    bc[l] += sum * pow(sc, l);
  }
}

/* Full 2D FMM.  classical = 0: shift-free passes; classical = 1: the textbook
 * method with M2M / L2L shifts.  Targets: tgt[0..nt) or all particles when tgt is
 * NULL.  Optional per-level dumps (level dump_k): moments and locals of every
 * box at that level (row-major boxes, P complex each). */
/* level_p (optional, [L + 1]): the order used at level k (P2M, M2L and L2P of
 * that level all truncate at level_p[k]); NULL means p at every level.  The
 * levels do not exchange coefficients in the shift-free method, so each level
 * is simply the fixed-order method of its own order.  Not with classical. */
int oracle_fmm2d_ex(int64_t n, const double* pos, const double* q, int L, int p, double side,
                    const double* origin, int classical, int64_t nt, const int64_t* tgt,
                    double* pot, double* field, int dump_k, double* dump_moments,
                    double* dump_locals, double* pot_far, double* pot_near,
                    const int* level_p) {
  if (n < 0 || L < 0 || L > 12 || p < 0 || p > 30 || !(side > 0)) return ORC_EINVAL;
  int pk[13];
  for (int k = 0; k <= L; ++k) {
    pk[k] = level_p ? level_p[k] : p;
    if (k >= 2 && (pk[k] < 0 || pk[k] > 30)) return ORC_EINVAL;
  }
  if (level_p && classical) return ORC_EINVAL;
  if (check_domain(2, n, pos, origin, side)) return ORC_EDOMAIN;
  if (!tgt) nt = n;
  tree t;
  if (tree_build(&t, 2, n, pos, origin, side, L)) return ORC_ENOMEM;
  int P = p + 1;
  cplx** A = calloc((size_t)L + 1, sizeof(cplx*));
  cplx** B = calloc((size_t)L + 1, sizeof(cplx*));
  for (int k = 2; k <= L; ++k) {
    int64_t nbox = ((int64_t)1 << k) * ((int64_t)1 << k);
    A[k] = calloc((size_t)(nbox * (pk[k] + 1)), sizeof(cplx));
    B[k] = calloc((size_t)(nbox * (pk[k] + 1)), sizeof(cplx));
    if (!A[k] || !B[k]) return ORC_ENOMEM;
  }
  /* which target boxes need locals */
  char** want = calloc((size_t)L + 1, sizeof(char*));
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k;
    want[k] = calloc((size_t)(nb * nb), 1);
    if (tgt == NULL || classical || k == dump_k) {
      memset(want[k], 1, (size_t)(nb * nb));
    } else {
      for (int64_t e = 0; e < nt; ++e) {
        const int64_t* c = &t.lc[2 * tgt[e]];
        want[k][(c[1] >> (L - k)) * nb + (c[0] >> (L - k))] = 1;
      }
    }
  }

  if (!classical) {
    /* U-bar: box vectors at every level straight from the particles. */
    for (int k = 2; k <= L; ++k) p2m2d_level(&t, pos, q, k, pk[k], side, origin, A[k]);
    /* D-bar-1: bilinear forms over the interaction list at every level. */
    for (int k = 2; k <= L; ++k) m2l2d_level(k, pk[k], side, A[k], want[k], B[k]);
  } else if (L >= 2) {
    /* U-1 at the finest level, U-2 shifts upward. */
    p2m2d_level(&t, pos, q, L, p, side, origin, A[L]);
    for (int k = L - 1; k >= 2; --k) {
      int64_t nb = (int64_t)1 << k;
      double sp = side / (double)nb, sc = sp / 2;
      for (int64_t c = 0; c < 4 * nb * nb; ++c) {
        int64_t cx = c % (2 * nb), cy = c / (2 * nb);
        m2m2d_one(p, sc, box_centre2d(origin, sc, cx, cy), sp,
                  box_centre2d(origin, sp, cx >> 1, cy >> 1), &A[k + 1][c * P],
                  &A[k][((cy >> 1) * nb + (cx >> 1)) * P]);
      }
    }
    /* D-1 at every level, D-2 shifts downward (accumulated into B). */
    for (int k = 2; k <= L; ++k) m2l2d_level(k, p, side, A[k], NULL, B[k]);
    for (int k = 2; k < L; ++k) {
      int64_t nb = (int64_t)1 << k;
      double sp = side / (double)nb, sc = sp / 2;
      for (int64_t c = 0; c < 4 * nb * nb; ++c) {
        int64_t cx = c % (2 * nb), cy = c / (2 * nb);
        l2l2d_one(p, sp, box_centre2d(origin, sp, cx >> 1, cy >> 1), sc,
                  box_centre2d(origin, sc, cx, cy), &B[k][((cy >> 1) * nb + (cx >> 1)) * P],
                  &B[k + 1][c * P]);
      }
    }
  }

  if (dump_k >= 2 && dump_k <= L) {
    int64_t nbox = ((int64_t)1 << dump_k) * ((int64_t)1 << dump_k);
    for (int64_t i = 0; i < nbox * (pk[dump_k] + 1); ++i) {
      if (dump_moments) {
        dump_moments[2 * i] = creal(A[dump_k][i]);
        dump_moments[2 * i + 1] = cimag(A[dump_k][i]);
      }
      if (dump_locals) {
        dump_locals[2 * i] = creal(B[dump_k][i]);
        dump_locals[2 * i + 1] = cimag(B[dump_k][i]);
      }
    }
  }

  /* Evaluation: far field from every level's local (shift-free) or from the
   * finest level's accumulated local (classical), plus the near field. */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < nt; ++e) {
    int64_t i = tgt ? tgt[e] : e;
    double x = pos[2 * i], y = pos[2 * i + 1];
    double far = 0, ef[2] = {0, 0};
    int klo = classical ? L : 2;
    for (int k = klo; k <= L && k >= 2; ++k) {
      int64_t nb = (int64_t)1 << k;
      double s = side / (double)nb;
      int64_t bx = t.lc[2 * i] >> (L - k), by = t.lc[2 * i + 1] >> (L - k);
      const int Pk = pk[k] + 1;
      l2p2d_one(pk[k], s, box_centre2d(origin, s, bx, by), &B[k][(by * nb + bx) * Pk], x, y,
                &far, ef);
    }
    double near, en[3];
    near_field(&t, pos, q, i, &near, en);
    pot[e] = near + far;
    if (field) {
      field[2 * e] = en[0] + ef[0];
      field[2 * e + 1] = en[1] + ef[1];
    }
    if (pot_far) pot_far[e] = far;
    if (pot_near) pot_near[e] = near;
  }

  for (int k = 2; k <= L; ++k) {
    free(A[k]);
    free(B[k]);
    free(want[k]);
  }
  free(A);
  free(B);
  free(want);
  tree_free(&t);
  return ORC_OK;
}

int oracle_fmm2d(int64_t n, const double* pos, const double* q, int L, int p, double side,
                 const double* origin, int classical, int64_t nt, const int64_t* tgt,
                 double* pot, double* field) {
  return oracle_fmm2d_ex(n, pos, q, L, p, side, origin, classical, nt, tgt, pot, field, -1, NULL,
                         NULL, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------- */
/* Adaptive depth (2D).  The paper's tree is uniform; for clustered inputs a   */
/* particle's tree may stop early.  In the shift-free passes every level's    */
/* box vectors come from the particles, so a particle whose leaf lies at      */
/* level d(i) simply runs the uniform method of depth d(i): the forms of its  */
/* ancestors' interaction lists at levels 2..d(i) (D-bar-1, D-bar-2 summed    */
/* over those levels) plus the direct sum over the particles of the 3 x 3     */
/* boxes around its level-d(i) box.  For each particle these sets partition  */
/* all other particles, exactly as for the uniform tree of depth d(i)         */
/* (Section 2.1, items 1-5), whatever d(i) is.  The depth bounds the direct   */
/* sum:                                                                       */
/*   d(i) = the first level k >= 2 at which the 3 x 3 boxes around the        */
/*          particle's level-k box hold at most near_max particles, and L if  */
/*          there is none.                                                    */
/* Those counts only fall with k, so all particles of a level-k box agree on  */
/* whether their depth reaches k.                                             */
/* ------------------------------------------------------------------------- */

/* Particles of the 3 x 3 boxes at level d around particle i's level-d box,
 * j != i, r > 0; boxes visited row by row, each box's leaves row by row. */
static void near_field_level2d(const tree* t, const double* pos, const double* q, int64_t i,
                               int d, double* phi, double* e) {
  int64_t span = (int64_t)1 << (t->L - d), nb = (int64_t)1 << d;
  int64_t cx = t->lc[2 * i] >> (t->L - d), cy = t->lc[2 * i + 1] >> (t->L - d);
  double ph = 0, ex = 0, ey = 0;
  for (int64_t by = cy - 1; by <= cy + 1; ++by)
    for (int64_t bx = cx - 1; bx <= cx + 1; ++bx) {
      if (bx < 0 || by < 0 || bx >= nb || by >= nb) continue;
      for (int64_t ly = by * span; ly < (by + 1) * span; ++ly)
        for (int64_t lx = bx * span; lx < (bx + 1) * span; ++lx) {
          int64_t lf = ly * t->nl + lx;
          for (int64_t s = t->start[lf]; s < t->start[lf + 1]; ++s) {
            int64_t j = t->idx[s];
            if (j == i) continue;
            double dx = pos[2 * i] - pos[2 * j], dy = pos[2 * i + 1] - pos[2 * j + 1];
            double r2 = dx * dx + dy * dy;
            if (r2 == 0.0) continue;
            ph += q[j] * 0.5 * log(r2);
            ex -= q[j] * dx / r2;
            ey -= q[j] * dy / r2;
          }
        }
    }
  *phi = ph;
  e[0] = ex;
  e[1] = ey;
}

int oracle_fmm2d_adaptive(int64_t n, const double* pos, const double* q, int L, int p,
                          int64_t near_max, double side, const double* origin, double* pot,
                          double* field, int32_t* depth) {
  if (n < 0 || L < 2 || L > 12 || p < 0 || p > 30 || near_max < 0 || !(side > 0))
    return ORC_EINVAL;
  if (check_domain(2, n, pos, origin, side)) return ORC_EDOMAIN;
  tree t;
  if (tree_build(&t, 2, n, pos, origin, side, L)) return ORC_ENOMEM;
  int P = p + 1;
  /* particle counts of every box at every level, from the leaves up */
  int64_t** cnt = calloc((size_t)L + 1, sizeof(int64_t*));
  cplx** A = calloc((size_t)L + 1, sizeof(cplx*));
  cplx** B = calloc((size_t)L + 1, sizeof(cplx*));
  char** want = calloc((size_t)L + 1, sizeof(char*));
  int* d = malloc(sizeof(int) * (size_t)(n + 1));
  if (!cnt || !A || !B || !want || !d) return ORC_ENOMEM;
  for (int k = 0; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k;
    cnt[k] = calloc((size_t)(nb * nb), sizeof(int64_t));
    if (!cnt[k]) return ORC_ENOMEM;
  }
  for (int64_t lf = 0; lf < t.nleaf; ++lf) cnt[L][lf] = t.start[lf + 1] - t.start[lf];
  for (int k = L - 1; k >= 0; --k) {
    int64_t nb = (int64_t)1 << k;
    for (int64_t b = 0; b < nb * nb; ++b) {
      int64_t bx = b % nb, by = b / nb;
      for (int c = 0; c < 4; ++c)
        cnt[k][b] += cnt[k + 1][(2 * by + (c >> 1)) * (2 * nb) + 2 * bx + (c & 1)];
    }
  }
  /* leaf depth of every particle, and the boxes whose locals it reads */
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k;
    A[k] = calloc((size_t)(nb * nb * P), sizeof(cplx));
    B[k] = calloc((size_t)(nb * nb * P), sizeof(cplx));
    want[k] = calloc((size_t)(nb * nb), 1);
    if (!A[k] || !B[k] || !want[k]) return ORC_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    int k = 2;
    for (;; ++k) {
      int64_t nb = (int64_t)1 << k;
      int64_t bx = t.lc[2 * i] >> (L - k), by = t.lc[2 * i + 1] >> (L - k), around = 0;
      for (int64_t y = by - 1; y <= by + 1; ++y)
        for (int64_t x = bx - 1; x <= bx + 1; ++x)
          if (x >= 0 && y >= 0 && x < nb && y < nb) around += cnt[k][y * nb + x];
      if (k == L || around <= near_max) break;
    }
    d[i] = k;
    if (depth) depth[i] = k;
    for (int kk = 2; kk <= k; ++kk) {
      int64_t nb = (int64_t)1 << kk;
      want[kk][(t.lc[2 * i + 1] >> (L - kk)) * nb + (t.lc[2 * i] >> (L - kk))] = 1;
    }
  }
  /* U-bar: box vectors at every level from the particles; D-bar-1 for the
   * boxes some particle reads */
  for (int k = 2; k <= L; ++k) p2m2d_level(&t, pos, q, k, p, side, origin, A[k]);
  for (int k = 2; k <= L; ++k) m2l2d_level(k, p, side, A[k], want[k], B[k]);
  /* D-bar-2 over levels 2..d(i), and the near field at level d(i) */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double x = pos[2 * i], y = pos[2 * i + 1];
    double far = 0, ef[2] = {0, 0};
    for (int k = 2; k <= d[i]; ++k) {
      int64_t nb = (int64_t)1 << k;
      double s = side / (double)nb;
      int64_t bx = t.lc[2 * i] >> (L - k), by = t.lc[2 * i + 1] >> (L - k);
      l2p2d_one(p, s, box_centre2d(origin, s, bx, by), &B[k][(by * nb + bx) * P], x, y, &far,
                ef);
    }
    double near, en[2];
    near_field_level2d(&t, pos, q, i, d[i], &near, en);
    pot[i] = near + far;
    if (field) {
      field[2 * i] = en[0] + ef[0];
      field[2 * i + 1] = en[1] + ef[1];
    }
  }
  for (int k = 0; k <= L; ++k) {
    free(cnt[k]);
    if (k >= 2) {
      free(A[k]);
      free(B[k]);
      free(want[k]);
    }
  }
  free(cnt);
  free(A);
  free(B);
  free(want);
  free(d);
  tree_free(&t);
  return ORC_OK;
}

/* Single-box check helpers for the truncation pins: moments of a set of charges
 * about centre (cx, cy) with scale s, and evaluation of the multipole series at
 * a far point.  */
int oracle_p2m2d_point(int64_t n, const double* pos, const double* q, double cx, double cy,
                       double s, int p, double* out /* [p+1][2] */) {
  cplx a[64] = {0};
  cplx zb = CMPLX(cx, cy);
  for (int64_t c = 0; c < n; ++c) {
    cplx w = (CMPLX(pos[2 * c], pos[2 * c + 1]) - zb) / s;
    a[0] += q[c];
    cplx wm = 1.0;
    for (int m = 1; m <= p; ++m) {
      wm *= w;
      a[m] += -q[c] * wm / (double)m;
    }
  }
  for (int m = 0; m <= p; ++m) {
    out[2 * m] = creal(a[m]);
    out[2 * m + 1] = cimag(a[m]);
  }
  return ORC_OK;
}

double oracle_m2p2d_point(const double* a_in, int p, double cx, double cy, double s, double x,
                          double y) {
  cplx d = CMPLX(x, y) - CMPLX(cx, cy);
  cplx acc = CMPLX(a_in[0], a_in[1]) * clog(d);
  cplx r = s / d, rm = 1.0;
  for (int m = 1; m <= p; ++m) {
    rm *= r;
    acc += CMPLX(a_in[2 * m], a_in[2 * m + 1]) * rm;
  }
  return creal(acc);
}

/* ========================================================================= */
/* 3D: solid harmonics of degree <= p, scaled by box side.                    */
/*                                                                           */
/* With P_n^m the associated Legendre function including the Condon-Shortley */
/* phase (P_n^-m = (-1)^m (n-m)!/(n+m)! P_n^m):                               */
/*   R_n^m(r) = r^n P_n^m(cos t) e^{i m f} / (n+m)!        (regular)           */
/*   I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}    (irregular)         */
/* so that, for |y| < |x|:                                                    */
/*   1/|x - y|  = sum_{n,m} conj(R_n^m(y)) I_n^m(x)                           */
/*   R_n^m(x+y) = sum_{j,k} R_j^k(x) R_{n-j}^{m-k}(y)                         */
/*   I_j^k(x-y) = sum_{n,m} conj(R_n^m(y)) I_{j+n}^{k+m}(x)                   */
/* Box b (centre r_b, side s); w = (r - r_b)/s.                               */
/*   moments : M_n^m = sum q conj(R_n^m(w))                                   */
/*   locals  : potential near target centre r_t:                               */
/*             (1/s) sum_{j,k} L_j^k R_j^k((r - r_t)/s)                        */
/*   M2L     : L_j^k += (-1)^k sum_{n,m} (-1)^n M_n^m I_{j+n}^{m-k}(u),        */
/*             u = (r_b - r_t)/s (an integer vector)                           */
/* Arrays hold every order m in [-n, n] at index n*n + n + m.                  */
/* ========================================================================= */

static int shi(int n, int m) { return n * n + n + m; }

/* Regular harmonics R_n^m(x, y, z), n <= p, by the Cartesian recurrences
 *   R_m^m = -(x + i y) / (2m) R_{m-1}^{m-1}
 *   (n - m)(n + m) R_n^m = (2n - 1) z R_{n-1}^m - r^2 R_{n-2}^m
 * (both follow from the Legendre recurrences), and R_n^-m = (-1)^m conj R_n^m. */
void oracle_sh_regular(int p, double x, double y, double z, double* out_ri) {
  cplx R[(64) * (64)];
  double r2 = x * x + y * y + z * z;
  cplx xy = CMPLX(x, y);
  R[shi(0, 0)] = 1.0;
  for (int m = 1; m <= p; ++m) R[shi(m, m)] = -xy / (2.0 * m) * R[shi(m - 1, m - 1)];
  for (int m = 0; m <= p; ++m)
    for (int n = m + 1; n <= p; ++n) {
      cplx prev2 = n - 2 >= m ? R[shi(n - 2, m)] : 0.0;
      R[shi(n, m)] = ((2.0 * n - 1.0) * z * R[shi(n - 1, m)] - r2 * prev2) /
                     ((double)(n - m) * (double)(n + m));
    }
  for (int n = 0; n <= p; ++n)
    for (int m = 1; m <= n; ++m) R[shi(n, -m)] = (m % 2 ? -1.0 : 1.0) * conj(R[shi(n, m)]);
  for (int i = 0; i < (p + 1) * (p + 1); ++i) {
    out_ri[2 * i] = creal(R[i]);
    out_ri[2 * i + 1] = cimag(R[i]);
  }
}

/* Irregular harmonics I_n^m(x, y, z), n <= p, by
 *   I_0^0 = 1/r,  I_m^m = -(2m - 1)(x + i y) / r^2 I_{m-1}^{m-1}
 *   r^2 I_n^m = (2n - 1) z I_{n-1}^m - (n + m - 1)(n - m - 1) I_{n-2}^m
 * and I_n^-m = (-1)^m conj I_n^m. */
void oracle_sh_irregular(int p, double x, double y, double z, double* out_ri) {
  cplx Ir[(64) * (64)];
  double r2 = x * x + y * y + z * z;
  cplx xy = CMPLX(x, y);
  Ir[shi(0, 0)] = 1.0 / sqrt(r2);
  for (int m = 1; m <= p; ++m) Ir[shi(m, m)] = -(2.0 * m - 1.0) * xy / r2 * Ir[shi(m - 1, m - 1)];
  for (int m = 0; m <= p; ++m)
    for (int n = m + 1; n <= p; ++n) {
      cplx prev2 = n - 2 >= m ? Ir[shi(n - 2, m)] : 0.0;
      Ir[shi(n, m)] = ((2.0 * n - 1.0) * z * Ir[shi(n - 1, m)] -
                      (double)(n + m - 1) * (double)(n - m - 1) * prev2) /
                     r2;
    }
  for (int n = 0; n <= p; ++n)
    for (int m = 1; m <= n; ++m) Ir[shi(n, -m)] = (m % 2 ? -1.0 : 1.0) * conj(Ir[shi(n, m)]);
  for (int i = 0; i < (p + 1) * (p + 1); ++i) {
    out_ri[2 * i] = creal(Ir[i]);
    out_ri[2 * i + 1] = cimag(Ir[i]);
  }
}

static void sh_reg_c(int p, double x, double y, double z, cplx* R) {
  double tmp[2 * 64 * 64];
  oracle_sh_regular(p, x, y, z, tmp);
  for (int i = 0; i < (p + 1) * (p + 1); ++i) R[i] = CMPLX(tmp[2 * i], tmp[2 * i + 1]);
}

static void sh_irr_c(int p, double x, double y, double z, cplx* Ir) {
  double tmp[2 * 64 * 64];
  oracle_sh_irregular(p, x, y, z, tmp);
  for (int i = 0; i < (p + 1) * (p + 1); ++i) Ir[i] = CMPLX(tmp[2 * i], tmp[2 * i + 1]);
}

static void box_centre3d(const double* o, double s, int64_t ix, int64_t iy, int64_t iz,
                         double* c) {
  c[0] = o[0] + s * ((double)ix + 0.5);
  c[1] = o[1] + s * ((double)iy + 0.5);
  c[2] = o[2] + s * ((double)iz + 0.5);
}

static void p2m3d_level(const tree* t, const double* pos, const double* q, int k, int p,
                        double side, const double* o, cplx* M) {
  int64_t nb = (int64_t)1 << k, span = (int64_t)1 << (t->L - k);
  double s = side / (double)nb;
  int NC = (p + 1) * (p + 1);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < nb * nb * nb; ++b) {
    int64_t bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
    double c[3];
    box_centre3d(o, s, bx, by, bz, c);
    cplx* mb = &M[b * NC];
    cplx R[64 * 64];
    for (int i = 0; i < NC; ++i) mb[i] = 0;
    for (int64_t lz = bz * span; lz < (bz + 1) * span; ++lz)
      for (int64_t ly = by * span; ly < (by + 1) * span; ++ly)
        for (int64_t lx = bx * span; lx < (bx + 1) * span; ++lx) {
          int64_t lf = (lz * t->nl + ly) * t->nl + lx;
          for (int64_t e = t->start[lf]; e < t->start[lf + 1]; ++e) {
            int64_t i = t->idx[e];
            sh_reg_c(p, (pos[3 * i] - c[0]) / s, (pos[3 * i + 1] - c[1]) / s,
                     (pos[3 * i + 2] - c[2]) / s, R);
            for (int n = 0; n <= p; ++n)
              for (int m = -n; m <= n; ++m) mb[shi(n, m)] += q[i] * conj(R[shi(n, m)]);
          }
        }
  }
}

static void m2l3d_one(int p, const double* u, const cplx* Mb, cplx* Lt) {
  cplx Ir[64 * 64];
  sh_irr_c(2 * p, u[0], u[1], u[2], Ir);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0;
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
          if (abs(m - k) > j + n) continue;
          acc += (n % 2 ? -1.0 : 1.0) * Mb[shi(n, m)] * Ir[shi(j + n, m - k)];
        }
      Lt[shi(j, k)] += (abs(k) % 2 ? -1.0 : 1.0) * acc;
    }
}

static void m2l3d_level(int k, int p, const cplx* M, const char* want, cplx* Lc) {
  int64_t nb = (int64_t)1 << k;
  int NC = (p + 1) * (p + 1);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < nb * nb * nb; ++t) {
    cplx* lt = &Lc[t * NC];
    for (int i = 0; i < NC; ++i) lt[i] = 0;
    if (want && !want[t]) continue;
    int64_t tx = t % nb, ty = (t / nb) % nb, tz = t / (nb * nb), il[3 * 189];
    int n = oracle_ilist3d(k, tx, ty, tz, il);
    for (int i = 0; i < n; ++i) {
      double u[3] = {(double)(il[3 * i] - tx), (double)(il[3 * i + 1] - ty),
                     (double)(il[3 * i + 2] - tz)};
      m2l3d_one(p, u, &M[((il[3 * i + 2] * nb + il[3 * i + 1]) * nb + il[3 * i]) * NC], lt);
    }
  }
}

/* Potential (1/s) sum L_j^k R_j^k(w) and field -grad, using
 *   d/dz R_j^k = R_{j-1}^k,  (d/dx + i d/dy) R_j^k = R_{j-1}^{k+1},
 *   (d/dx - i d/dy) R_j^k = -R_{j-1}^{k-1}. */
static void l2p3d_one(int p, double s, const double* c, const cplx* Lt, const double* r,
                      double* phi, double* e) {
  cplx R[64 * 64];
  double w[3] = {(r[0] - c[0]) / s, (r[1] - c[1]) / s, (r[2] - c[2]) / s};
  sh_reg_c(p, w[0], w[1], w[2], R);
  cplx f = 0, gx = 0, gy = 0, gz = 0;
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx L = Lt[shi(j, k)];
      f += L * R[shi(j, k)];
      if (j == 0) continue;
      cplx up = abs(k + 1) <= j - 1 ? R[shi(j - 1, k + 1)] : 0.0;
      cplx dn = abs(k - 1) <= j - 1 ? R[shi(j - 1, k - 1)] : 0.0;
      cplx zz = abs(k) <= j - 1 ? R[shi(j - 1, k)] : 0.0;
      gz += L * zz;
      gx += L * 0.5 * (up - dn);
      gy += L * (up + dn) / CMPLX(0.0, 2.0);
    }
  *phi += creal(f) / s;
  e[0] += -creal(gx) / (s * s);
  e[1] += -creal(gy) / (s * s);
  e[2] += -creal(gz) / (s * s);
}

/* Classical shifts, unscaled.  M2M: a child multipole about r_c moved to the
 * parent centre r_p with d = r_c - r_p:  M_n^m += sum_{j,k} M_j^k conj R_{n-j}^{m-k}(d).
 * L2L: a parent local moved to a child centre:  L_n^m += sum_{j>=n,k} L_j^k R_{j-n}^{k-m}(d). */
static void m2m3d_one(int p, double sc, const double* cc, double sp, const double* cp,
                      const cplx* Mc, cplx* Mp) {
  cplx R[64 * 64];
  sh_reg_c(p, cc[0] - cp[0], cc[1] - cp[1], cc[2] - cp[2], R);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      cplx acc = 0;
      for (int j = 0; j <= n; ++j)
        for (int k = -j; k <= j; ++k) {
          if (abs(m - k) > n - j) continue;
          acc += Mc[shi(j, k)] * pow(sc, j) * conj(R[shi(n - j, m - k)]);
        }
      Mp[shi(n, m)] += acc / pow(sp, n);
    }
}

static void l2l3d_one(int p, double sp, const double* cp, double sc, const double* cc,
                      const cplx* Lp, cplx* Lc) {
  cplx R[64 * 64];
  sh_reg_c(p, cc[0] - cp[0], cc[1] - cp[1], cc[2] - cp[2], R);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      cplx acc = 0;
      for (int j = n; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
          if (abs(k - m) > j - n) continue;
          acc += Lp[shi(j, k)] / pow(sp, j + 1) * R[shi(j - n, k - m)];
        }
      Lc[shi(n, m)] += acc * pow(sc, n + 1);
    }
}

int oracle_fmm3d_ex(int64_t n, const double* pos, const double* q, int L, int p, double side,
                    const double* origin, int classical, int64_t nt, const int64_t* tgt,
                    double* pot, double* field, int dump_k, double* dump_moments,
                    double* dump_locals) {
  if (n < 0 || L < 0 || L > 8 || p < 0 || p > 20 || !(side > 0)) return ORC_EINVAL;
  if (check_domain(3, n, pos, origin, side)) return ORC_EDOMAIN;
  if (!tgt) nt = n;
  tree t;
  if (tree_build(&t, 3, n, pos, origin, side, L)) return ORC_ENOMEM;
  int NC = (p + 1) * (p + 1);
  cplx** M = calloc((size_t)L + 1, sizeof(cplx*));
  cplx** Lc = calloc((size_t)L + 1, sizeof(cplx*));
  char** want = calloc((size_t)L + 1, sizeof(char*));
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k, nbox = nb * nb * nb;
    M[k] = calloc((size_t)(nbox * NC), sizeof(cplx));
    Lc[k] = calloc((size_t)(nbox * NC), sizeof(cplx));
    want[k] = calloc((size_t)nbox, 1);
    if (!M[k] || !Lc[k] || !want[k]) return ORC_ENOMEM;
    if (tgt == NULL || classical || k == dump_k) {
      memset(want[k], 1, (size_t)nbox);
    } else {
      for (int64_t e = 0; e < nt; ++e) {
        const int64_t* c = &t.lc[3 * tgt[e]];
        want[k][((c[2] >> (L - k)) * nb + (c[1] >> (L - k))) * nb + (c[0] >> (L - k))] = 1;
      }
    }
  }
  if (!classical) {
    for (int k = 2; k <= L; ++k) p2m3d_level(&t, pos, q, k, p, side, origin, M[k]);
    for (int k = 2; k <= L; ++k) m2l3d_level(k, p, M[k], want[k], Lc[k]);
  } else if (L >= 2) {
    p2m3d_level(&t, pos, q, L, p, side, origin, M[L]);
    for (int k = L - 1; k >= 2; --k) {
      int64_t nb = (int64_t)1 << k;
      double sp = side / (double)nb, sc = sp / 2;
      for (int64_t c = 0; c < 8 * nb * nb * nb; ++c) {
        int64_t cx = c % (2 * nb), cy = (c / (2 * nb)) % (2 * nb), cz = c / (4 * nb * nb);
        double cc[3], cp[3];
        box_centre3d(origin, sc, cx, cy, cz, cc);
        box_centre3d(origin, sp, cx >> 1, cy >> 1, cz >> 1, cp);
        m2m3d_one(p, sc, cc, sp, cp, &M[k + 1][c * NC],
                  &M[k][(((cz >> 1) * nb + (cy >> 1)) * nb + (cx >> 1)) * NC]);
      }
    }
    for (int k = 2; k <= L; ++k) m2l3d_level(k, p, M[k], NULL, Lc[k]);
    for (int k = 2; k < L; ++k) {
      int64_t nb = (int64_t)1 << k;
      double sp = side / (double)nb, sc = sp / 2;
      for (int64_t c = 0; c < 8 * nb * nb * nb; ++c) {
        int64_t cx = c % (2 * nb), cy = (c / (2 * nb)) % (2 * nb), cz = c / (4 * nb * nb);
        double cc[3], cp[3];
        box_centre3d(origin, sc, cx, cy, cz, cc);
        box_centre3d(origin, sp, cx >> 1, cy >> 1, cz >> 1, cp);
        l2l3d_one(p, sp, cp, sc, cc, &Lc[k][(((cz >> 1) * nb + (cy >> 1)) * nb + (cx >> 1)) * NC],
                  &Lc[k + 1][c * NC]);
      }
    }
  }
  if (dump_k >= 2 && dump_k <= L) {
    int64_t nb = (int64_t)1 << dump_k, nbox = nb * nb * nb;
    for (int64_t i = 0; i < nbox * NC; ++i) {
      if (dump_moments) {
        dump_moments[2 * i] = creal(M[dump_k][i]);
        dump_moments[2 * i + 1] = cimag(M[dump_k][i]);
      }
      if (dump_locals) {
        dump_locals[2 * i] = creal(Lc[dump_k][i]);
        dump_locals[2 * i + 1] = cimag(Lc[dump_k][i]);
      }
    }
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < nt; ++e) {
    int64_t i = tgt ? tgt[e] : e;
    double far = 0, ef[3] = {0, 0, 0};
    int klo = classical ? L : 2;
    for (int k = klo; k <= L && k >= 2; ++k) {
      int64_t nb = (int64_t)1 << k;
      double s = side / (double)nb, c[3];
      int64_t bx = t.lc[3 * i] >> (L - k), by = t.lc[3 * i + 1] >> (L - k),
              bz = t.lc[3 * i + 2] >> (L - k);
      box_centre3d(origin, s, bx, by, bz, c);
      l2p3d_one(p, s, c, &Lc[k][((bz * nb + by) * nb + bx) * NC], &pos[3 * i], &far, ef);
    }
    double near, en[3];
    near_field(&t, pos, q, i, &near, en);
    pot[e] = near + far;
    if (field) {
      field[3 * e] = en[0] + ef[0];
      field[3 * e + 1] = en[1] + ef[1];
      field[3 * e + 2] = en[2] + ef[2];
    }
  }
  for (int k = 2; k <= L; ++k) {
    free(M[k]);
    free(Lc[k]);
    free(want[k]);
  }
  free(M);
  free(Lc);
  free(want);
  tree_free(&t);
  return ORC_OK;
}

/* ========================================================================= */
/* 3D with the paper's own realisation of V: fixed point charges (Appendix,  */
/* STEP1-STEP5).  In every box, n points per axis at the offsets a_i * s / 5  */
/* from the centre (s = box side; the paper's set is n = 4, a = {-2, -1, 1, 2}, */
/* and any distinct offsets may be chosen, Fig. 3's caption), d = n^3 points, */
/* point (i, j, l) (x, y, z offsets a_i, a_j, a_l) at index i + n j + n^2 l.   */
/*   STEP2 (h_m): a charge q at x in box m becomes the d point charges         */
/*     q f_i(u_x) f_j(u_y) f_l(u_z),  u = 5 (x - centre) / s,                 */
/*     f_i(u) = prod_{k != i} (u - a_k) / (a_i - a_k)  (Lagrange, in units s/5);*/
/*     summed over the box's charges this is the box vector (its moments).    */
/*   STEP3 (b_{m1,m2}): the bilinear form of two well-separated boxes is the  */
/*     pair sum of their point charges, sum_{i,j} c1_i c2_j / |y1_i - y2_j|;  */
/*     the linear form of a target box (its locals) is therefore             */
/*     L_i = sum_{m2 in IL} sum_j M_j(m2) / |y_i(t) - y_j(m2)|.               */
/*   The potential of a charge at x in the target box is sum_i f_i(u) L_i, the */
/*   same map h applied to the probe charge (D-bar-2: summed over levels).    */
/* Everything is formed per level straight from the particles (shift-free);   */
/* the root-frame form of STEP4-STEP5 follows further below.                  */
/* ========================================================================= */
#define LAG_MAXN 8

typedef struct {
  int n;                 /* points per axis */
  double a[LAG_MAXN];    /* their offsets from the centre, in units of s / 5 */
} lagset;

static const lagset kPaperNodes = {4, {-2.0, -1.0, 1.0, 2.0}};

static int lagset_make(int np, const double* nodes, lagset* S) {
  if (np < 1 || np > LAG_MAXN || !nodes) return ORC_EINVAL;
  S->n = np;
  for (int i = 0; i < np; ++i) {
    if (!isfinite(nodes[i])) return ORC_EINVAL;
    for (int k = 0; k < i; ++k)
      if (nodes[k] == nodes[i]) return ORC_EINVAL;  /* distinct nodes (eq. (1)) */
    S->a[i] = nodes[i];
  }
  return ORC_OK;
}

/* f_i(u) as the quotient F_i(u) / F_i(a_i) of the STEP2 interpolation formula. */
static double lag_f(const lagset* S, int i, double u) {
  double num = 1.0, den = 1.0;
  for (int k = 0; k < S->n; ++k) {
    if (k == i) continue;
    num *= u - S->a[k];
    den *= S->a[i] - S->a[k];
  }
  return num / den;
}

/* d f_i / du: the product rule over the n - 1 factors of F_i. */
static double lag_df(const lagset* S, int i, double u) {
  double den = 1.0, sum = 0.0;
  for (int k = 0; k < S->n; ++k)
    if (k != i) den *= S->a[i] - S->a[k];
  for (int drop = 0; drop < S->n; ++drop) {
    if (drop == i) continue;
    double prod = 1.0;
    for (int k = 0; k < S->n; ++k)
      if (k != i && k != drop) prod *= u - S->a[k];
    sum += prod;
  }
  return sum / den;
}

void oracle_lagrange_weights(double u, double* f, double* df) {
  for (int i = 0; i < 4; ++i) {
    f[i] = lag_f(&kPaperNodes, i, u);
    df[i] = lag_df(&kPaperNodes, i, u);
  }
}

/* The same for any node set (np nodes, offsets in units of s / 5). */
int oracle_lagrange_weights_nodes(int np, const double* nodes, double u, double* f, double* df) {
  lagset S;
  if (lagset_make(np, nodes, &S)) return ORC_EINVAL;
  for (int i = 0; i < np; ++i) {
    f[i] = lag_f(&S, i, u);
    df[i] = lag_df(&S, i, u);
  }
  return ORC_OK;
}

/* Physical position of point `idx` of box (bx, by, bz) at level side s. */
static void lag_point(const lagset* S, const double* o, double s, int64_t bx, int64_t by,
                      int64_t bz, int idx, double* y) {
  double c[3];
  int n = S->n;
  box_centre3d(o, s, bx, by, bz, c);
  y[0] = c[0] + S->a[idx % n] * s / 5.0;
  y[1] = c[1] + S->a[(idx / n) % n] * s / 5.0;
  y[2] = c[2] + S->a[idx / (n * n)] * s / 5.0;
}

/* h_m(x) of a unit charge at x for the box of side s centred at c: the d
 * weights f_i(u_x) f_j(u_y) f_l(u_z) (STEP2), and with grad != NULL their
 * gradients in x (chain rule du/dx = 5 / s), [d][3]. */
static void lag_weights3(const lagset* S, double s, const double* c, const double* x, double* w,
                         double* grad) {
  int n = S->n;
  double f[3][LAG_MAXN], df[3][LAG_MAXN];
  for (int d = 0; d < 3; ++d) {
    double u = 5.0 * (x[d] - c[d]) / s;
    for (int a = 0; a < n; ++a) {
      f[d][a] = lag_f(S, a, u);
      df[d][a] = lag_df(S, a, u);
    }
  }
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j)
      for (int a = 0; a < n; ++a) {
        int idx = a + n * j + n * n * l;
        w[idx] = f[0][a] * f[1][j] * f[2][l];
        if (grad) {
          grad[3 * idx] = df[0][a] * f[1][j] * f[2][l] * 5.0 / s;
          grad[3 * idx + 1] = f[0][a] * df[1][j] * f[2][l] * 5.0 / s;
          grad[3 * idx + 2] = f[0][a] * f[1][j] * df[2][l] * 5.0 / s;
        }
      }
}

/* STEP2 summed over each box of level k: M[b * d + idx]. */
static void lagp2m_level(const lagset* S, const tree* t, const double* pos, const double* q, int k,
                         double side, const double* o, double* M) {
  int n = S->n, d = n * n * n;
  int64_t nb = (int64_t)1 << k;
  double s = side / (double)nb;
  for (int64_t b = 0; b < nb * nb * nb; ++b) {
    for (int i = 0; i < d; ++i) M[b * d + i] = 0.0;
  }
  int64_t np = t->start[t->nleaf];
  for (int64_t e = 0; e < np; ++e) {
    int64_t i = t->idx[e];
    int64_t bx = t->lc[3 * i] >> (t->L - k), by = t->lc[3 * i + 1] >> (t->L - k),
            bz = t->lc[3 * i + 2] >> (t->L - k);
    double c[3];
    box_centre3d(o, s, bx, by, bz, c);
    double fx[LAG_MAXN], fy[LAG_MAXN], fz[LAG_MAXN];
    for (int a = 0; a < n; ++a) {
      fx[a] = lag_f(S, a, 5.0 * (pos[3 * i] - c[0]) / s);
      fy[a] = lag_f(S, a, 5.0 * (pos[3 * i + 1] - c[1]) / s);
      fz[a] = lag_f(S, a, 5.0 * (pos[3 * i + 2] - c[2]) / s);
    }
    double* mb = &M[((bz * nb + by) * nb + bx) * d];
    for (int l = 0; l < n; ++l)
      for (int j = 0; j < n; ++j)
        for (int a = 0; a < n; ++a) mb[a + n * j + n * n * l] += q[i] * fx[a] * fy[j] * fz[l];
  }
}

/* STEP3 linear forms of the marked boxes of level k. */
static void lagm2l_level(const lagset* S, int k, double side, const double* o, const double* M,
                         const char* want, double* Lc) {
  int d = S->n * S->n * S->n;
  int64_t nb = (int64_t)1 << k;
  double s = side / (double)nb;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t b = 0; b < nb * nb * nb; ++b) {
    double* lb = &Lc[b * d];
    for (int i = 0; i < d; ++i) lb[i] = 0.0;
    if (want && !want[b]) continue;
    int64_t tx = b % nb, ty = (b / nb) % nb, tz = b / (nb * nb);
    int64_t il[3 * 189];
    int cnt = oracle_ilist3d(k, tx, ty, tz, il);
    for (int e = 0; e < cnt; ++e) {
      const double* ms = &M[((il[3 * e + 2] * nb + il[3 * e + 1]) * nb + il[3 * e]) * d];
      for (int i = 0; i < d; ++i) {
        double yi[3];
        lag_point(S, o, s, tx, ty, tz, i, yi);
        double acc = 0.0;
        for (int j = 0; j < d; ++j) {
          double yj[3];
          lag_point(S, o, s, il[3 * e], il[3 * e + 1], il[3 * e + 2], j, yj);
          double dx = yi[0] - yj[0], dy = yi[1] - yj[1], dz = yi[2] - yj[2];
          acc += ms[j] / sqrt(dx * dx + dy * dy + dz * dz);
        }
        lb[i] += acc;
      }
    }
  }
}

/* Probe charge at x in box (bx, by, bz): potential sum_i f_i L_i and its
 * negative gradient (chain rule du/dx = 5 / s). */
static void lagl2p_one(const lagset* S, double s, const double* c, const double* lb,
                       const double* x, double* phi, double* e) {
  int n = S->n;
  double u[3], f[3][LAG_MAXN], df[3][LAG_MAXN];
  for (int d = 0; d < 3; ++d) {
    u[d] = 5.0 * (x[d] - c[d]) / s;
    for (int a = 0; a < n; ++a) {
      f[d][a] = lag_f(S, a, u[d]);
      df[d][a] = lag_df(S, a, u[d]);
    }
  }
  double ph = 0, gx = 0, gy = 0, gz = 0;
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j)
      for (int a = 0; a < n; ++a) {
        double v = lb[a + n * j + n * n * l];
        ph += f[0][a] * f[1][j] * f[2][l] * v;
        gx += df[0][a] * f[1][j] * f[2][l] * v;
        gy += f[0][a] * df[1][j] * f[2][l] * v;
        gz += f[0][a] * f[1][j] * df[2][l] * v;
      }
  *phi += ph;
  e[0] -= gx * 5.0 / s;
  e[1] -= gy * 5.0 / s;
  e[2] -= gz * 5.0 / s;
}

/* Full evaluation with the point-charge basis of node set S (levels 2..L,
 * near field over the 27 leaves).  dump_k >= 2: moments / locals of every box
 * of that level, [nbox][d] each (row-major box order, x fastest). */
static int lagrange_eval(const lagset* S, int64_t n, const double* pos, const double* q, int L,
                         double side, const double* origin, int64_t nt, const int64_t* tgt,
                         double* pot, double* field, int dump_k, double* dump_moments,
                         double* dump_locals) {
  if (n < 0 || L < 0 || L > 6 || !(side > 0)) return ORC_EINVAL;
  if (check_domain(3, n, pos, origin, side)) return ORC_EDOMAIN;
  int d = S->n * S->n * S->n;
  if (!tgt) nt = n;
  tree t;
  if (tree_build(&t, 3, n, pos, origin, side, L)) return ORC_ENOMEM;
  double** M = calloc((size_t)L + 1, sizeof(double*));
  double** Lc = calloc((size_t)L + 1, sizeof(double*));
  char** want = calloc((size_t)L + 1, sizeof(char*));
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k, nbox = nb * nb * nb;
    M[k] = calloc((size_t)(nbox * d), sizeof(double));
    Lc[k] = calloc((size_t)(nbox * d), sizeof(double));
    want[k] = calloc((size_t)nbox, 1);
    if (!M[k] || !Lc[k] || !want[k]) return ORC_ENOMEM;
    if (tgt == NULL || k == dump_k) {
      memset(want[k], 1, (size_t)nbox);
    } else {
      for (int64_t e = 0; e < nt; ++e) {
        const int64_t* c = &t.lc[3 * tgt[e]];
        want[k][((c[2] >> (L - k)) * nb + (c[1] >> (L - k))) * nb + (c[0] >> (L - k))] = 1;
      }
    }
  }
  for (int k = 2; k <= L; ++k) lagp2m_level(S, &t, pos, q, k, side, origin, M[k]);
  for (int k = 2; k <= L; ++k) lagm2l_level(S, k, side, origin, M[k], want[k], Lc[k]);
  if (dump_k >= 2 && dump_k <= L) {
    int64_t nb = (int64_t)1 << dump_k, nbox = nb * nb * nb;
    if (dump_moments) memcpy(dump_moments, M[dump_k], sizeof(double) * (size_t)(nbox * d));
    if (dump_locals) memcpy(dump_locals, Lc[dump_k], sizeof(double) * (size_t)(nbox * d));
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < nt; ++e) {
    int64_t i = tgt ? tgt[e] : e;
    double far = 0, ef[3] = {0, 0, 0};
    for (int k = 2; k <= L; ++k) {
      int64_t nb = (int64_t)1 << k;
      double s = side / (double)nb, c[3];
      int64_t bx = t.lc[3 * i] >> (L - k), by = t.lc[3 * i + 1] >> (L - k),
              bz = t.lc[3 * i + 2] >> (L - k);
      box_centre3d(origin, s, bx, by, bz, c);
      lagl2p_one(S, s, c, &Lc[k][((bz * nb + by) * nb + bx) * d], &pos[3 * i], &far, ef);
    }
    double near, en[3];
    near_field(&t, pos, q, i, &near, en);
    pot[e] = near + far;
    if (field) {
      field[3 * e] = en[0] + ef[0];
      field[3 * e + 1] = en[1] + ef[1];
      field[3 * e + 2] = en[2] + ef[2];
    }
  }
  for (int k = 2; k <= L; ++k) {
    free(M[k]);
    free(Lc[k]);
    free(want[k]);
  }
  free(M);
  free(Lc);
  free(want);
  tree_free(&t);
  return ORC_OK;
}

/* The paper's node set: n = 4 at {-2, -1, 1, 2}. */
int oracle_fmm3d_lagrange(int64_t n, const double* pos, const double* q, int L, double side,
                          const double* origin, int64_t nt, const int64_t* tgt, double* pot,
                          double* field, int dump_k, double* dump_moments, double* dump_locals) {
  return lagrange_eval(&kPaperNodes, n, pos, q, L, side, origin, nt, tgt, pot, field, dump_k,
                       dump_moments, dump_locals);
}

/* Any node set: np nodes per axis at offsets nodes[] (units of s / 5). */
int oracle_fmm3d_lagrange_nodes(int np, const double* nodes, int64_t n, const double* pos,
                                const double* q, int L, double side, const double* origin,
                                int64_t nt, const int64_t* tgt, double* pot, double* field,
                                int dump_k, double* dump_moments, double* dump_locals) {
  lagset S;
  if (lagset_make(np, nodes, &S)) return ORC_EINVAL;
  return lagrange_eval(&S, n, pos, q, L, side, origin, nt, tgt, pot, field, dump_k, dump_moments,
                       dump_locals);
}

/* ========================================================================= */
/* 2D with the paper's point charges (Appendix STEP1 and Fig. 3 describe the  */
/* square box with n = 4 points per axis, d = 16), the log kernel.  Point      */
/* (i, j) (x, y offsets a_i, a_j in units of s / 5) at index i + n j.          */
/*   STEP2: a charge q at x in box m becomes the d point charges              */
/*     q f_i(u_x) f_j(u_y),  u = 5 (x - centre) / s;                          */
/*   STEP3: the bilinear form of two well-separated boxes is the pair sum     */
/*     sum_{a,b} c1_a c2_b log|y1_a - y2_b|, so the linear form (locals) of   */
/*     a target box is L_a = sum_{m2 in IL} sum_b M_b(m2) log|y_a - y_b(m2)|;  */
/*   the potential of a probe at x in the box is sum_a f(u) L_a (the same map  */
/*   h), its field minus the gradient of that in x; summed over levels.       */
/* ========================================================================= */
static void lag_point2(const lagset* S, const double* o, double s, int64_t bx, int64_t by,
                       int idx, double* y) {
  cplx c = box_centre2d(o, s, bx, by);
  y[0] = creal(c) + S->a[idx % S->n] * s / 5.0;
  y[1] = cimag(c) + S->a[idx / S->n] * s / 5.0;
}

/* STEP2 summed over each box of level k: M[b * d + idx], b = by * 2^k + bx. */
static void lagp2m_level2d(const lagset* S, const tree* t, const double* pos, const double* q,
                           int k, double side, const double* o, double* M) {
  int n = S->n, d = n * n;
  int64_t nb = (int64_t)1 << k;
  double s = side / (double)nb;
  for (int64_t e = 0; e < nb * nb * d; ++e) M[e] = 0.0;
  int64_t np = t->start[t->nleaf];
  for (int64_t e = 0; e < np; ++e) {
    int64_t i = t->idx[e];
    int64_t bx = t->lc[2 * i] >> (t->L - k), by = t->lc[2 * i + 1] >> (t->L - k);
    cplx c = box_centre2d(o, s, bx, by);
    double fx[LAG_MAXN], fy[LAG_MAXN];
    for (int a = 0; a < n; ++a) {
      fx[a] = lag_f(S, a, 5.0 * (pos[2 * i] - creal(c)) / s);
      fy[a] = lag_f(S, a, 5.0 * (pos[2 * i + 1] - cimag(c)) / s);
    }
    double* mb = &M[(by * nb + bx) * d];
    for (int j = 0; j < n; ++j)
      for (int a = 0; a < n; ++a) mb[a + n * j] += q[i] * fx[a] * fy[j];
  }
}

/* STEP3 linear forms of the marked boxes of level k. */
static void lagm2l_level2d(const lagset* S, int k, double side, const double* o, const double* M,
                           const char* want, double* Lc) {
  int d = S->n * S->n;
  int64_t nb = (int64_t)1 << k;
  double s = side / (double)nb;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t b = 0; b < nb * nb; ++b) {
    double* lb = &Lc[b * d];
    for (int i = 0; i < d; ++i) lb[i] = 0.0;
    if (want && !want[b]) continue;
    int64_t tx = b % nb, ty = b / nb;
    int64_t il[2 * 27];
    int cnt = oracle_ilist2d(k, tx, ty, il);
    for (int e = 0; e < cnt; ++e) {
      const double* ms = &M[(il[2 * e + 1] * nb + il[2 * e]) * d];
      for (int i = 0; i < d; ++i) {
        double yi[2];
        lag_point2(S, o, s, tx, ty, i, yi);
        double acc = 0.0;
        for (int j = 0; j < d; ++j) {
          double yj[2];
          lag_point2(S, o, s, il[2 * e], il[2 * e + 1], j, yj);
          double dx = yi[0] - yj[0], dy = yi[1] - yj[1];
          acc += ms[j] * 0.5 * log(dx * dx + dy * dy);
        }
        lb[i] += acc;
      }
    }
  }
}

/* Probe charge at x in the box of side s centred at c: potential sum_a f L_a
 * and its negative gradient (chain rule du/dx = 5 / s). */
static void lagl2p_one2d(const lagset* S, double s, cplx c, const double* lb, const double* x,
                         double* phi, double* e) {
  int n = S->n;
  double fx[LAG_MAXN], fy[LAG_MAXN], dfx[LAG_MAXN], dfy[LAG_MAXN];
  double ux = 5.0 * (x[0] - creal(c)) / s, uy = 5.0 * (x[1] - cimag(c)) / s;
  for (int a = 0; a < n; ++a) {
    fx[a] = lag_f(S, a, ux);
    dfx[a] = lag_df(S, a, ux);
    fy[a] = lag_f(S, a, uy);
    dfy[a] = lag_df(S, a, uy);
  }
  double ph = 0, gx = 0, gy = 0;
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < n; ++a) {
      double v = lb[a + n * j];
      ph += fx[a] * fy[j] * v;
      gx += dfx[a] * fy[j] * v;
      gy += fx[a] * dfy[j] * v;
    }
  *phi += ph;
  e[0] -= gx * 5.0 / s;
  e[1] -= gy * 5.0 / s;
}

/* Full 2D evaluation with the point-charge basis of node set S (levels 2..L,
 * near field over the 9 leaves).  dump_k >= 2: moments / locals of every box of
 * that level, [nbox][d] each (row-major box order, x fastest). */
static int lagrange_eval2d(const lagset* S, int64_t n, const double* pos, const double* q, int L,
                           double side, const double* origin, int64_t nt, const int64_t* tgt,
                           double* pot, double* field, int dump_k, double* dump_moments,
                           double* dump_locals) {
  if (n < 0 || L < 0 || L > 9 || !(side > 0)) return ORC_EINVAL;
  if (check_domain(2, n, pos, origin, side)) return ORC_EDOMAIN;
  int d = S->n * S->n;
  if (!tgt) nt = n;
  tree t;
  if (tree_build(&t, 2, n, pos, origin, side, L)) return ORC_ENOMEM;
  double** M = calloc((size_t)L + 1, sizeof(double*));
  double** Lc = calloc((size_t)L + 1, sizeof(double*));
  char** want = calloc((size_t)L + 1, sizeof(char*));
  if (!M || !Lc || !want) return ORC_ENOMEM;
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k, nbox = nb * nb;
    M[k] = calloc((size_t)(nbox * d), sizeof(double));
    Lc[k] = calloc((size_t)(nbox * d), sizeof(double));
    want[k] = calloc((size_t)nbox, 1);
    if (!M[k] || !Lc[k] || !want[k]) return ORC_ENOMEM;
    if (tgt == NULL || k == dump_k) {
      memset(want[k], 1, (size_t)nbox);
    } else {
      for (int64_t e = 0; e < nt; ++e) {
        const int64_t* c = &t.lc[2 * tgt[e]];
        want[k][(c[1] >> (L - k)) * nb + (c[0] >> (L - k))] = 1;
      }
    }
  }
  for (int k = 2; k <= L; ++k) lagp2m_level2d(S, &t, pos, q, k, side, origin, M[k]);
  for (int k = 2; k <= L; ++k) lagm2l_level2d(S, k, side, origin, M[k], want[k], Lc[k]);
  if (dump_k >= 2 && dump_k <= L) {
    int64_t nb = (int64_t)1 << dump_k, nbox = nb * nb;
    if (dump_moments) memcpy(dump_moments, M[dump_k], sizeof(double) * (size_t)(nbox * d));
    if (dump_locals) memcpy(dump_locals, Lc[dump_k], sizeof(double) * (size_t)(nbox * d));
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < nt; ++e) {
    int64_t i = tgt ? tgt[e] : e;
    double far = 0, ef[2] = {0, 0};
    for (int k = 2; k <= L; ++k) {
      int64_t nb = (int64_t)1 << k;
      double s = side / (double)nb;
      int64_t bx = t.lc[2 * i] >> (L - k), by = t.lc[2 * i + 1] >> (L - k);
      lagl2p_one2d(S, s, box_centre2d(origin, s, bx, by), &Lc[k][(by * nb + bx) * d],
                   &pos[2 * i], &far, ef);
    }
    double near, en[2];
    near_field(&t, pos, q, i, &near, en);
    pot[e] = near + far;
    if (field) {
      field[2 * e] = en[0] + ef[0];
      field[2 * e + 1] = en[1] + ef[1];
    }
  }
  for (int k = 2; k <= L; ++k) {
    free(M[k]);
    free(Lc[k]);
    free(want[k]);
  }
  free(M);
  free(Lc);
  free(want);
  tree_free(&t);
  return ORC_OK;
}

/* 2D, any node set: np nodes per axis at offsets nodes[] (units of s / 5). */
int oracle_fmm2d_lagrange_nodes(int np, const double* nodes, int64_t n, const double* pos,
                                const double* q, int L, double side, const double* origin,
                                int64_t nt, const int64_t* tgt, double* pot, double* field,
                                int dump_k, double* dump_moments, double* dump_locals) {
  lagset S;
  if (lagset_make(np, nodes, &S)) return ORC_EINVAL;
  return lagrange_eval2d(&S, n, pos, q, L, side, origin, nt, tgt, pot, field, dump_k,
                         dump_moments, dump_locals);
}

/* ========================================================================= */
/* The root-frame passes of Section 2.2.1 with the point-charge V, as the     */
/* paper writes them (Appendix STEP4-STEP5):                                  */
/*   V = the values of the d point charges of the root box m^0; a particle c  */
/*     maps to v = h_{m^0}(c) (STEP2 in the root box, the same for every box  */
/*     containing c: the Note closing Section 2.2.2);                         */
/*   U-bar-1: v_{m^l} = sum of v over the particles of each finest box;       */
/*   U-bar-2: v_{m^k} = sum of the v of its 8 children, k = l-1 .. 2;         */
/*   STEP4: M_m = (h_m(p_1), ..., h_m(p_d)), p_j the unit point charges of    */
/*     m^0: it carries a root-frame vector to the d charges of box m;         */
/*   STEP3/STEP5: B_{mi,m}(v_k, v_l) = b_{mi,m}(M_mi v_k, M_m v_l), b the pair */
/*     sum of point charges (M_b[a][j] = 1 / |y_a(mi) - y_j(m)|);             */
/*   D-bar-1: L~_m(v) = sum_{mi in IL(m)} B_{mi,m}(v_mi, v) at every level     */
/*     2..l, kept as the dual vector M_m^T M_b^T M_mi v_mi summed over IL(m);  */
/*   D-bar-2: L_{m^2} = L~_{m^2} (levels 0 and 1 carry no list), then          */
/*     L_child = L~_child + L_parent down to level l;                          */
/*   F(v) = L_{m^l}(v): the far potential of a unit probe at x is             */
/*     L_{m^l} . h_{m^0}(x), its field minus the gradient of that in x.       */
/* In exact arithmetic M_m h_{m^0}(c) = h_m(c) (eq. (1): the root weights      */
/* reproduce every polynomial of degree < n, and h_m is one), so this equals  */
/* the box-local form above.  In floating point the entries of M_m grow with  */
/* the level (h_m evaluated at root points far outside m), which is why the   */
/* paper asks for double precision (Discussion (3)); *max_transfer receives  */
/* the largest |entry| of any M_m used.                                       */
/* ========================================================================= */

/* STEP4 for box (bx, by, bz) of level k: M[i * d + j] = h_m(p_j)[i]. */
static void lag_transfer(const lagset* S, double side, const double* o, int k, int64_t bx,
                         int64_t by, int64_t bz, double* M) {
  int d = S->n * S->n * S->n;
  double s = side / (double)((int64_t)1 << k), c[3], w[LAG_MAXN * LAG_MAXN * LAG_MAXN];
  box_centre3d(o, s, bx, by, bz, c);
  for (int j = 0; j < d; ++j) {
    double pj[3];
    lag_point(S, o, side, 0, 0, 0, j, pj);  /* root point p_j */
    lag_weights3(S, s, c, pj, w, NULL);     /* h_m(p_j) */
    for (int i = 0; i < d; ++i) M[i * d + j] = w[i];
  }
}

int oracle_lagrange_transfer(int np, const double* nodes, double side, const double* origin,
                             int k, int64_t bx, int64_t by, int64_t bz, double* M) {
  lagset S;
  if (lagset_make(np, nodes, &S) || k < 0) return ORC_EINVAL;
  lag_transfer(&S, side, origin, k, bx, by, bz, M);
  return ORC_OK;
}

/* h_m(x) of a unit charge for box (bx, by, bz) of level k (level 0: the root). */
int oracle_lagrange_box_weights(int np, const double* nodes, double side, const double* origin,
                                int k, int64_t bx, int64_t by, int64_t bz, const double* x,
                                double* w) {
  lagset S;
  if (lagset_make(np, nodes, &S) || k < 0) return ORC_EINVAL;
  double s = side / (double)((int64_t)1 << k), c[3];
  box_centre3d(origin, s, bx, by, bz, c);
  lag_weights3(&S, s, c, x, w, NULL);
  return ORC_OK;
}

int oracle_fmm3d_lagrange_root(int np, const double* nodes, int64_t n, const double* pos,
                               const double* q, int L, double side, const double* origin,
                               int64_t nt, const int64_t* tgt, double* pot, double* field,
                               double* max_transfer) {
  lagset S;
  if (lagset_make(np, nodes, &S)) return ORC_EINVAL;
  if (n < 0 || L < 0 || L > 4 || !(side > 0)) return ORC_EINVAL;
  if (check_domain(3, n, pos, origin, side)) return ORC_EDOMAIN;
  const int d = S.n * S.n * S.n;
  if (!tgt) nt = n;
  tree t;
  if (tree_build(&t, 3, n, pos, origin, side, L)) return ORC_ENOMEM;
  double croot[3];
  box_centre3d(origin, side, 0, 0, 0, croot);
  double** V = calloc((size_t)L + 1, sizeof(double*));   /* v_m, root frame */
  double** Lt = calloc((size_t)L + 1, sizeof(double*));  /* L~_m, dual, root frame */
  double** Lf = calloc((size_t)L + 1, sizeof(double*));  /* L_m after D-bar-2 */
  double** Mt = calloc((size_t)L + 1, sizeof(double*));  /* M_m of every box */
  if (!V || !Lt || !Lf || !Mt) return ORC_ENOMEM;
  for (int k = 2; k <= L; ++k) {
    int64_t nb = (int64_t)1 << k, nbox = nb * nb * nb;
    V[k] = calloc((size_t)(nbox * d), sizeof(double));
    Lt[k] = calloc((size_t)(nbox * d), sizeof(double));
    Lf[k] = calloc((size_t)(nbox * d), sizeof(double));
    Mt[k] = calloc((size_t)(nbox * d * d), sizeof(double));
    if (!V[k] || !Lt[k] || !Lf[k] || !Mt[k]) return ORC_ENOMEM;
  }
  double mt = 0.0;
  if (L >= 2) {
    /* U-bar-1: each particle's root-frame vector added into its finest box */
    int64_t nb = (int64_t)1 << L;
    for (int64_t e = 0; e < n; ++e) {
      double w[LAG_MAXN * LAG_MAXN * LAG_MAXN];
      lag_weights3(&S, side, croot, &pos[3 * e], w, NULL); /* h_{m^0}(c) / q */
      const int64_t* c = &t.lc[3 * e];
      double* vb = &V[L][((c[2] * nb + c[1]) * nb + c[0]) * d];
      for (int i = 0; i < d; ++i) vb[i] += q[e] * w[i];
    }
    /* U-bar-2: coarser boxes as sums of their children */
    for (int k = L - 1; k >= 2; --k) {
      int64_t nb2 = (int64_t)1 << k, nf = nb2 * 2;
      for (int64_t bz = 0; bz < nb2; ++bz)
        for (int64_t by = 0; by < nb2; ++by)
          for (int64_t bx = 0; bx < nb2; ++bx) {
            double* vb = &V[k][((bz * nb2 + by) * nb2 + bx) * d];
            for (int cz = 0; cz < 2; ++cz)
              for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                  const double* vc =
                      &V[k + 1][(((2 * bz + cz) * nf + 2 * by + cy) * nf + 2 * bx + cx) * d];
                  for (int i = 0; i < d; ++i) vb[i] += vc[i];
                }
          }
    }
    /* STEP4: M_m of every box at levels 2..l */
    for (int k = 2; k <= L; ++k) {
      int64_t nb2 = (int64_t)1 << k;
#pragma omp parallel for schedule(dynamic, 4)
      for (int64_t b = 0; b < nb2 * nb2 * nb2; ++b)
        lag_transfer(&S, side, origin, k, b % nb2, (b / nb2) % nb2, b / (nb2 * nb2),
                     &Mt[k][b * d * d]);
      for (int64_t e = 0; e < nb2 * nb2 * nb2 * d * d; ++e)
        if (fabs(Mt[k][e]) > mt) mt = fabs(Mt[k][e]);
    }
    /* D-bar-1 at every level 2..l */
    for (int k = 2; k <= L; ++k) {
      int64_t nb2 = (int64_t)1 << k;
      double s = side / (double)nb2;
#pragma omp parallel for schedule(dynamic, 4)
      for (int64_t b = 0; b < nb2 * nb2 * nb2; ++b) {
        int64_t tx = b % nb2, ty = (b / nb2) % nb2, tz = b / (nb2 * nb2);
        int64_t il[3 * 189];
        int cnt = oracle_ilist3d(k, tx, ty, tz, il);
        double* lt = &Lt[k][b * d];
        const double* Mm = &Mt[k][b * d * d];
        double* u = malloc(sizeof(double) * (size_t)d);
        double* y = malloc(sizeof(double) * (size_t)d);
        for (int e = 0; e < cnt; ++e) {
          int64_t sb = (il[3 * e + 2] * nb2 + il[3 * e + 1]) * nb2 + il[3 * e];
          const double* Mi = &Mt[k][sb * d * d];
          const double* vi = &V[k][sb * d];
          /* u = M_mi v_mi: the source box's charges */
          for (int a = 0; a < d; ++a) {
            double acc = 0.0;
            for (int j = 0; j < d; ++j) acc += Mi[a * d + j] * vi[j];
            u[a] = acc;
          }
          /* y = M_b^T u: the potentials at the target box's points */
          for (int j = 0; j < d; ++j) {
            double yj[3], acc = 0.0;
            lag_point(&S, origin, s, tx, ty, tz, j, yj);
            for (int a = 0; a < d; ++a) {
              double ya[3];
              lag_point(&S, origin, s, il[3 * e], il[3 * e + 1], il[3 * e + 2], a, ya);
              double dx = ya[0] - yj[0], dy = ya[1] - yj[1], dz = ya[2] - yj[2];
              acc += u[a] / sqrt(dx * dx + dy * dy + dz * dz);
            }
            y[j] = acc;
          }
          /* L~_m += M_m^T y: back to the root frame */
          for (int r = 0; r < d; ++r) {
            double acc = 0.0;
            for (int j = 0; j < d; ++j) acc += Mm[j * d + r] * y[j];
            lt[r] += acc;
          }
        }
        free(u);
        free(y);
      }
    }
    /* D-bar-2: parent-to-child additions of the dual vectors */
    for (int k = 2; k <= L; ++k) {
      int64_t nb2 = (int64_t)1 << k, nbp = nb2 / 2;
      for (int64_t b = 0; b < nb2 * nb2 * nb2; ++b) {
        double* lf = &Lf[k][b * d];
        const double* lt = &Lt[k][b * d];
        if (k == 2) {
          for (int i = 0; i < d; ++i) lf[i] = lt[i];
        } else {
          int64_t tx = b % nb2, ty = (b / nb2) % nb2, tz = b / (nb2 * nb2);
          const double* lp = &Lf[k - 1][(((tz >> 1) * nbp + (ty >> 1)) * nbp + (tx >> 1)) * d];
          for (int i = 0; i < d; ++i) lf[i] = lt[i] + lp[i];
        }
      }
    }
  }
  /* F(v) = L_{m^l}(v) at each target, plus the near field */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < nt; ++e) {
    int64_t i = tgt ? tgt[e] : e;
    double far = 0, ef[3] = {0, 0, 0};
    if (L >= 2) {
      double w[LAG_MAXN * LAG_MAXN * LAG_MAXN], g[3 * LAG_MAXN * LAG_MAXN * LAG_MAXN];
      lag_weights3(&S, side, croot, &pos[3 * i], w, g);
      int64_t nb = (int64_t)1 << L;
      const int64_t* c = &t.lc[3 * i];
      const double* lf = &Lf[L][((c[2] * nb + c[1]) * nb + c[0]) * d];
      for (int r = 0; r < d; ++r) {
        far += lf[r] * w[r];
        ef[0] -= lf[r] * g[3 * r];
        ef[1] -= lf[r] * g[3 * r + 1];
        ef[2] -= lf[r] * g[3 * r + 2];
      }
    }
    double near, en[3];
    near_field(&t, pos, q, i, &near, en);
    pot[e] = near + far;
    if (field) {
      field[3 * e] = en[0] + ef[0];
      field[3 * e + 1] = en[1] + ef[1];
      field[3 * e + 2] = en[2] + ef[2];
    }
  }
  if (max_transfer) *max_transfer = mt;
  for (int k = 2; k <= L; ++k) {
    free(V[k]);
    free(Lt[k]);
    free(Lf[k]);
    free(Mt[k]);
  }
  free(V);
  free(Lt);
  free(Lf);
  free(Mt);
  tree_free(&t);
  return ORC_OK;
}
