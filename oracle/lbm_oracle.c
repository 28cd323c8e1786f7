/*
 * lbm_oracle.c -- plain, slow, FP64 reference of the D3Q19 BGK lattice
 * Boltzmann update (Habich et al., "Performance engineering for the Lattice
 * Boltzmann method on GPGPUs", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source, header, table
 * or helper with the HIP path: the velocity set below is generated here by
 * enumeration, the population layout inside the oracle is array-of-structures
 * in enumeration order, streaming is a push (the GPU path pulls), and the
 * adjoint is an explicit 19x19 Jacobian (the GPU path uses a rank-structured
 * closed form).
 *
 * Conventions (all FP64):
 *   - Public arrays use the interface layout: populations [19][nz][ny][nx]
 *     in interface direction order (table ABI_E below, matched to the
 *     internal enumeration by velocity vector), scalar fields [nz][ny][nx],
 *     vector fields [3][nz][ny][nx].
 *   - The stored state after n steps is the post-collision field f*(n).
 *     One step: stream f*(n) (with half-way bounce-back at solid neighbours),
 *     then collide every fluid cell.  f*(0) = f^eq(rho0, u0).
 *   - All axes are periodic.  flags: bit0 = solid, bit1 = no body force,
 *     bit2 = moving wall (a solid cell that moves with the velocity wall_u).
 *   - Body force: Guo, Zheng & Shi (Phys. Rev. E 65, 046308, 2002), with F
 *     a force density, applied on fluid cells without the no-force bit.
 *   - Moving walls: the half-way bounce-back of a link into a moving solid
 *     cell is corrected by the momentum the wall imparts (Ladd, J. Fluid
 *     Mech. 271, 285, 1994), with the reference density rho0 = 1.
 *   - Two equilibria (the `incompressible` argument): 0 = the second-order
 *     LBGK equilibrium of Qian et al. with u = j/rho (the default); 1 = the
 *     incompressible variant of He & Luo (J. Stat. Phys. 88, 927, 1997)
 *     with u = j/rho0, rho0 = 1, which the paper's "incompressible flow
 *     solver" (abstract, Sec. 2) may refer to.
 *
 * Every function names the passage of the paper (or the outside method) it
 * follows.  The paper defers the equilibrium to Qian et al. (1992); the
 * second-order LBGK equilibrium is written out in equilibrium() below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define FLAG_SOLID 1u
#define FLAG_NOFORCE 2u
#define FLAG_MOVING 4u

/* ---------------------------------------------------------------------- */
/* Lattice: Sec. 2 -- D3Q19, 19 discrete velocities in 3-D (Qian 1992).    */
/* Generated: every c in {-1,0,1}^3 with |c|^2 <= 2, weights by |c|^2.     */
/* ---------------------------------------------------------------------- */
static int C[Q][3];
static double W[Q];
static int OPP[Q];
static int ABI2INT[Q]; /* interface index -> internal index */
static int lattice_ready = 0;

/* Interface direction order of the population arrays (an interface
 * convention, not a property of the method). */
static const int ABI_E[Q][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int lattice_init(void) {
  if (lattice_ready) return 0;
  int q = 0;
  for (int cz = -1; cz <= 1; ++cz)
    for (int cy = -1; cy <= 1; ++cy)
      for (int cx = -1; cx <= 1; ++cx) {
        int n2 = cx * cx + cy * cy + cz * cz;
        if (n2 > 2) continue;
        C[q][0] = cx;
        C[q][1] = cy;
        C[q][2] = cz;
        W[q] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        ++q;
      }
  if (q != Q) return -1;
  for (int a = 0; a < Q; ++a) {
    OPP[a] = -1;
    for (int b = 0; b < Q; ++b)
      if (C[b][0] == -C[a][0] && C[b][1] == -C[a][1] && C[b][2] == -C[a][2])
        OPP[a] = b;
    if (OPP[a] < 0) return -1;
  }
  for (int k = 0; k < Q; ++k) {
    ABI2INT[k] = -1;
    for (int a = 0; a < Q; ++a)
      if (C[a][0] == ABI_E[k][0] && C[a][1] == ABI_E[k][1] &&
          C[a][2] == ABI_E[k][2])
        ABI2INT[k] = a;
    if (ABI2INT[k] < 0) return -1;
  }
  lattice_ready = 1;
  return 0;
}

/* Export the lattice in interface order, for the tests. */
int oracle_lattice(int *e /*[19][3]*/, double *w /*[19]*/, int *opp /*[19]*/) {
  if (lattice_init()) return -1;
  int int2abi[Q];
  for (int k = 0; k < Q; ++k) int2abi[ABI2INT[k]] = k;
  for (int k = 0; k < Q; ++k) {
    int a = ABI2INT[k];
    for (int d = 0; d < 3; ++d) e[3 * k + d] = C[a][d];
    w[k] = W[a];
    opp[k] = int2abi[OPP[a]];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Single-cell physics (internal order).                                  */
/* ---------------------------------------------------------------------- */

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double cdot(int i, const double *v) {
  return C[i][0] * v[0] + C[i][1] * v[1] + C[i][2] * v[2];
}

/* Sec. 2 step 2: second-order LBGK equilibrium of Qian et al. (1992) with
 * c_s^2 = 1/3:  f^eq_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u].
 * Incompressible variant (He & Luo 1997), rho0 = 1:
 *               f^eq_i = w_i [rho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]. */
static void equilibrium(double rho, const double *u, int incomp, double *feq) {
  double uu = dot3(u, u);
  for (int i = 0; i < Q; ++i) {
    double cu = cdot(i, u);
    double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    feq[i] = incomp ? W[i] * (rho + poly) : W[i] * rho * (1.0 + poly);
  }
}

/* The velocity of a cell from its moments: u = (j + F/2)/rho, or with the
 * incompressible equilibrium u = (j + F/2)/rho0, rho0 = 1. */
static void velocity(double rho, const double *j, const double *F, int incomp,
                     double *u) {
  for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / (incomp ? 1.0 : rho);
}

/* Guo et al. (2002) forcing term for BGK:
 * S_i = (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F */
static void guo_source(double omega, const double *u, const double *F,
                       double *S) {
  double uF = dot3(u, F);
  for (int i = 0; i < Q; ++i) {
    double cu = cdot(i, u);
    double cF = cdot(i, F);
    S[i] = (1.0 - 0.5 * omega) * W[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
  }
}

/* Sec. 2 steps 1-2 with Guo forcing: moments, equilibrium, relaxation.
 *   rho = sum f_i,  u = (sum f_i c_i + F/2) / rho   (/ rho0 if incomp),
 *   f*_i = f_i - (1/tau) (f_i - f^eq_i) + S_i. */
static void collide_cell(double omega, const double *F, int incomp,
                         const double *f, double *fout) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int d = 0; d < 3; ++d) j[d] += f[i] * C[i][d];
  }
  double u[3];
  velocity(rho, j, F, incomp, u);
  double feq[Q], S[Q];
  equilibrium(rho, u, incomp, feq);
  guo_source(omega, u, F, S);
  for (int i = 0; i < Q; ++i) fout[i] = f[i] - omega * (f[i] - feq[i]) + S[i];
}

/* Jacobians of the collision map of collide_cell, written out by the chain
 * rule (used by the discrete adjoint):
 *   J[i][j]  = d f*_i / d f_j,   JF[i][a] = d f*_i / d F_a.
 * d rho/d f_j = 1;  d u/d f_j = (c_j - u)/rho and d u/d F = I/(2 rho), or
 * with the incompressible equilibrium d u/d f_j = c_j and d u/d F = I/2. */
static void collide_jacobian(double omega, const double *F, int incomp,
                             const double *f, double J[Q][Q], double JF[Q][3]) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int d = 0; d < 3; ++d) j[d] += f[i] * C[i][d];
  }
  double u[3];
  velocity(rho, j, F, incomp, u);
  double uu = dot3(u, u);
  double rho_u = incomp ? 1.0 : rho; /* the density that divides j in u */
  for (int i = 0; i < Q; ++i) {
    double cu = cdot(i, u), cF = cdot(i, F);
    double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    double dfeq_drho = incomp ? W[i] : W[i] * (1.0 + poly);
    double dfeq_du[3], dS_du[3], dS_dF[3];
    for (int a = 0; a < 3; ++a) {
      dfeq_du[a] = W[i] * rho_u * (3.0 * C[i][a] + 9.0 * cu * C[i][a] - 3.0 * u[a]);
      dS_du[a] = (1.0 - 0.5 * omega) * W[i] * (-3.0 * F[a] + 9.0 * cF * C[i][a]);
      dS_dF[a] = (1.0 - 0.5 * omega) * W[i] * (3.0 * (C[i][a] - u[a]) + 9.0 * cu * C[i][a]);
    }
    for (int jj = 0; jj < Q; ++jj) {
      double v = ((i == jj) ? (1.0 - omega) : 0.0) + omega * dfeq_drho;
      for (int a = 0; a < 3; ++a) {
        double du_df = incomp ? C[jj][a] : (C[jj][a] - u[a]) / rho;
        v += (omega * dfeq_du[a] + dS_du[a]) * du_df;
      }
      J[i][jj] = v;
    }
    for (int a = 0; a < 3; ++a)
      JF[i][a] = dS_dF[a] + (omega * dfeq_du[a] + dS_du[a]) / (2.0 * rho_u);
  }
}

/* Interface-order wrappers of the single-cell functions, for the tests. */
static void abi_to_int(const double *fa, double *fi) {
  for (int k = 0; k < Q; ++k) fi[ABI2INT[k]] = fa[k];
}
static void int_to_abi(const double *fi, double *fa) {
  for (int k = 0; k < Q; ++k) fa[k] = fi[ABI2INT[k]];
}

int oracle_equilibrium(double rho, const double *u, int incomp, double *feq_abi) {
  if (lattice_init()) return -1;
  double t[Q];
  equilibrium(rho, u, incomp, t);
  int_to_abi(t, feq_abi);
  return 0;
}

int oracle_guo_source(double omega, const double *u, const double *F,
                      double *S_abi) {
  if (lattice_init()) return -1;
  double t[Q];
  guo_source(omega, u, F, t);
  int_to_abi(t, S_abi);
  return 0;
}

int oracle_collide(double tau, const double *F, int incomp, const double *f_abi,
                   double *fstar_abi) {
  if (lattice_init()) return -1;
  double a[Q], b[Q];
  abi_to_int(f_abi, a);
  collide_cell(1.0 / tau, F, incomp, a, b);
  int_to_abi(b, fstar_abi);
  return 0;
}

/* J_abi[i][j] = d f*_i / d f_j, JF_abi[i][a] = d f*_i / d F_a (interface order). */
int oracle_collide_jacobian(double tau, const double *F, int incomp,
                            const double *f_abi, double *J_abi, double *JF_abi) {
  if (lattice_init()) return -1;
  double a[Q], J[Q][Q], JF[Q][3];
  abi_to_int(f_abi, a);
  collide_jacobian(1.0 / tau, F, incomp, a, J, JF);
  for (int k = 0; k < Q; ++k) {
    for (int l = 0; l < Q; ++l) J_abi[k * Q + l] = J[ABI2INT[k]][ABI2INT[l]];
    for (int d = 0; d < 3; ++d) JF_abi[k * 3 + d] = JF[ABI2INT[k]][d];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Grid helpers.                                                          */
/* ---------------------------------------------------------------------- */
typedef struct {
  int nx, ny, nz;
  long n;
} grid;

static long cell(const grid *g, int x, int y, int z) {
  return ((long)z * g->ny + y) * g->nx + x;
}
static int wrap(int v, int n) { return ((v % n) + n) % n; }
static int is_solid(const uint8_t *flags, long c) {
  return flags && (flags[c] & FLAG_SOLID);
}
static int is_moving(const uint8_t *flags, long c) {
  return flags && (flags[c] & FLAG_SOLID) && (flags[c] & FLAG_MOVING);
}
static void cell_force(const uint8_t *flags, long c, const double *F,
                       double *Fc) {
  int off = flags && (flags[c] & FLAG_NOFORCE);
  for (int d = 0; d < 3; ++d) Fc[d] = off ? 0.0 : F[d];
}

/* interface SoA [19][n] <-> internal AoS [n][19] */
static void load_abi(const grid *g, const double *src, double *dst) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g->n; ++c)
    for (int k = 0; k < Q; ++k) dst[c * Q + ABI2INT[k]] = src[(long)k * g->n + c];
}
static void store_abi(const grid *g, const double *src, double *dst) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g->n; ++c)
    for (int k = 0; k < Q; ++k) dst[(long)k * g->n + c] = src[c * Q + ABI2INT[k]];
}

static int check_dims(int nx, int ny, int nz) {
  return (nx < 1 || ny < 1 || nz < 1) ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Grid-level entry points.                                               */
/* ---------------------------------------------------------------------- */

/* Initial state f*(0) = f^eq(rho0, u0) on fluid cells, 0 on solid cells.
 * rho0 may be NULL (uniform 1), u0 may be NULL (rest). */
int oracle_init(int nx, int ny, int nz, const uint8_t *flags, int incomp,
                const double *rho0, const double *u0, double *f_abi) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *a = calloc((size_t)g.n * Q, sizeof(double));
  if (!a) return -2;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g.n; ++c) {
    if (is_solid(flags, c)) continue;
    double rho = rho0 ? rho0[c] : 1.0;
    double u[3] = {0.0, 0.0, 0.0};
    if (u0)
      for (int d = 0; d < 3; ++d) u[d] = u0[(long)d * g.n + c];
    equilibrium(rho, u, incomp, a + c * Q);
  }
  store_abi(&g, a, f_abi);
  free(a);
  return 0;
}

/* Sec. 2 step 3 with the bounce-back of the obstacle paragraph: push the
 * post-collision values of every fluid cell to the neighbour along c_i; a
 * value that would enter a solid cell returns to its own cell reversed
 * (half-way bounce-back).  If that solid cell is a moving wall, the returning
 * value loses 2 w_i rho0 (c_i.u_w)/c_s^2 = 6 w_i (c_i.u_w) (Ladd 1994,
 * rho0 = 1), so a wall moving along c_i sends less back against itself.
 * wall_u may be NULL (no moving walls).  dst must be zeroed by the caller. */
static void stream_push(const grid *g, const uint8_t *flags,
                        const double *wall_u, const double *src, double *dst) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->nz; ++z)
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        long c = cell(g, x, y, z);
        if (is_solid(flags, c)) continue;
        for (int i = 0; i < Q; ++i) {
          long t = cell(g, wrap(x + C[i][0], g->nx), wrap(y + C[i][1], g->ny),
                        wrap(z + C[i][2], g->nz));
          if (!is_solid(flags, t))
            dst[t * Q + i] = src[c * Q + i];
          else if (wall_u && is_moving(flags, t))
            dst[c * Q + OPP[i]] = src[c * Q + i] - 6.0 * W[i] * cdot(i, wall_u);
          else
            dst[c * Q + OPP[i]] = src[c * Q + i];
        }
      }
}

/* n full time steps of the two-lattice scheme (Sec. 2, last paragraph):
 * stream f*(t) into the second lattice, collide there, swap. */
int oracle_step(int nx, int ny, int nz, double tau, const double *F,
                const uint8_t *flags, const double *wall_u, int incomp,
                double *f_abi, long nsteps) {
  if (lattice_init() || check_dims(nx, ny, nz) || nsteps < 0) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double omega = 1.0 / tau;
  double *a = malloc((size_t)g.n * Q * sizeof(double));
  double *b = malloc((size_t)g.n * Q * sizeof(double));
  if (!a || !b) {
    free(a);
    free(b);
    return -2;
  }
  load_abi(&g, f_abi, a);
  for (long s = 0; s < nsteps; ++s) {
    memset(b, 0, (size_t)g.n * Q * sizeof(double));
    stream_push(&g, flags, wall_u, a, b);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < g.n; ++c) {
      if (is_solid(flags, c)) {
        for (int i = 0; i < Q; ++i) a[c * Q + i] = 0.0;
        continue;
      }
      double Fc[3];
      cell_force(flags, c, F, Fc);
      collide_cell(omega, Fc, incomp, b + c * Q, a + c * Q);
    }
  }
  store_abi(&g, a, f_abi);
  free(a);
  free(b);
  return 0;
}

/* Pure streaming with bounce-back (no collision), for the tests. */
int oracle_stream(int nx, int ny, int nz, const uint8_t *flags,
                  const double *wall_u, double *f_abi, long nsteps) {
  if (lattice_init() || check_dims(nx, ny, nz) || nsteps < 0) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *a = malloc((size_t)g.n * Q * sizeof(double));
  double *b = malloc((size_t)g.n * Q * sizeof(double));
  if (!a || !b) {
    free(a);
    free(b);
    return -2;
  }
  load_abi(&g, f_abi, a);
  for (long s = 0; s < nsteps; ++s) {
    memset(b, 0, (size_t)g.n * Q * sizeof(double));
    stream_push(&g, flags, wall_u, a, b);
    double *t = a;
    a = b;
    b = t;
  }
  store_abi(&g, a, f_abi);
  free(a);
  free(b);
  return 0;
}

/* Sec. 2 step 1, evaluated on the stored post-collision state:
 * rho = sum f*_i, rho u = sum f*_i c_i - F/2 (rho0 u with the incompressible
 * equilibrium, rho0 = 1; either way this equals the pre-collision (rho, u) of
 * the same step under Guo forcing).  Solid cells give 0. */
int oracle_macroscopics(int nx, int ny, int nz, const double *F,
                        const uint8_t *flags, int incomp, const double *f_abi,
                        double *rho, double *u) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g.n; ++c) {
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    if (!is_solid(flags, c)) {
      for (int k = 0; k < Q; ++k) {
        double fv = f_abi[(long)k * g.n + c];
        r += fv;
        for (int d = 0; d < 3; ++d) m[d] += fv * ABI_E[k][d];
      }
    }
    double Fc[3];
    cell_force(flags, c, F, Fc);
    if (rho) rho[c] = r;
    if (u)
      for (int d = 0; d < 3; ++d)
        u[(long)d * g.n + c] =
            is_solid(flags, c) ? 0.0 : (m[d] - 0.5 * Fc[d]) / (incomp ? 1.0 : r);
  }
  return 0;
}

/* Global mass, momentum and kinetic energy over fluid cells:
 * out = {sum rho, sum rho u_x, sum rho u_y, sum rho u_z, sum rho |u|^2 / 2},
 * with rho0 = 1 in place of rho in the last four for the incompressible
 * equilibrium (its momentum density is rho0 u). */
int oracle_reduce(int nx, int ny, int nz, const double *F, const uint8_t *flags,
                  int incomp, const double *f_abi, double *out5) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *rho = malloc((size_t)g.n * sizeof(double));
  double *u = malloc((size_t)g.n * 3 * sizeof(double));
  if (!rho || !u) {
    free(rho);
    free(u);
    return -2;
  }
  oracle_macroscopics(nx, ny, nz, F, flags, incomp, f_abi, rho, u);
  double s[5] = {0, 0, 0, 0, 0};
  for (long c = 0; c < g.n; ++c) {
    if (is_solid(flags, c)) continue;
    double uc[3] = {u[c], u[g.n + c], u[2 * g.n + c]};
    double m = incomp ? 1.0 : rho[c];
    s[0] += rho[c];
    for (int d = 0; d < 3; ++d) s[1 + d] += m * uc[d];
    s[4] += 0.5 * m * dot3(uc, uc);
  }
  for (int k = 0; k < 5; ++k) out5[k] = s[k];
  free(rho);
  free(u);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Discrete adjoint (reverse mode of the update above).  The objective L   */
/* depends on the final macroscopic fields; lambda^n = dL/d f*(n).         */
/* ---------------------------------------------------------------------- */

/* Seed: lambda^T_i = dL/drho + dL/du . (c_i - u)/rho on fluid cells (0 on
 * solid), from rho = sum f*, u = (sum f* c - F/2)/rho;  dLdF += -dL/du/(2 rho)
 * on forced fluid cells (accumulated into dLdF[3]).  With the incompressible
 * equilibrium u = sum f* c - F/2, so lambda^T_i = dL/drho + dL/du . c_i and
 * dLdF += -dL/du/2. */
int oracle_adjoint_seed(int nx, int ny, int nz, const double *F,
                        const uint8_t *flags, int incomp, const double *fT_abi,
                        const double *dL_drho, const double *dL_du,
                        double *lam_abi, double *dLdF) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *rho = malloc((size_t)g.n * sizeof(double));
  double *u = malloc((size_t)g.n * 3 * sizeof(double));
  if (!rho || !u) {
    free(rho);
    free(u);
    return -2;
  }
  oracle_macroscopics(nx, ny, nz, F, flags, incomp, fT_abi, rho, u);
  double acc[3] = {0, 0, 0};
  for (long c = 0; c < g.n; ++c) {
    if (is_solid(flags, c)) {
      for (int k = 0; k < Q; ++k) lam_abi[(long)k * g.n + c] = 0.0;
      continue;
    }
    double gr = dL_drho ? dL_drho[c] : 0.0;
    double gu[3] = {0, 0, 0};
    if (dL_du)
      for (int d = 0; d < 3; ++d) gu[d] = dL_du[(long)d * g.n + c];
    double uc[3] = {u[c], u[g.n + c], u[2 * g.n + c]};
    double rho_u = incomp ? 1.0 : rho[c];
    for (int k = 0; k < Q; ++k) {
      double v = gr;
      for (int d = 0; d < 3; ++d)
        v += gu[d] * (incomp ? ABI_E[k][d] : (ABI_E[k][d] - uc[d]) / rho[c]);
      lam_abi[(long)k * g.n + c] = v;
    }
    int forced = !(flags && (flags[c] & FLAG_NOFORCE));
    if (forced)
      for (int d = 0; d < 3; ++d) acc[d] += -gu[d] / (2.0 * rho_u);
  }
  for (int d = 0; d < 3; ++d) dLdF[d] += acc[d];
  free(rho);
  free(u);
  return 0;
}

/* The collision's part of a reverse step (internal layout): at every fluid
 * cell, mu = J(f)^T lambda, the transposed Jacobian of the collision at the
 * pre-collision state f (explicit 19x19 matrix of collide_jacobian), and
 * dLdF += JF(f)^T lambda on forced fluid cells; mu = 0 on solid cells. */
static int adjoint_collide_aos(const grid *g, double omega, const double *F,
                               const uint8_t *flags, int incomp, const double *f,
                               const double *lam, double *mu, double *dLdF) {
  double *dF = calloc((size_t)g->n * 3, sizeof(double));
  if (!dF) return -2;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g->n; ++c) {
    if (is_solid(flags, c)) {
      for (int i = 0; i < Q; ++i) mu[c * Q + i] = 0.0;
      continue;
    }
    double Fc[3], J[Q][Q], JF[Q][3];
    cell_force(flags, c, F, Fc);
    collide_jacobian(omega, Fc, incomp, f + c * Q, J, JF);
    for (int jj = 0; jj < Q; ++jj) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += lam[c * Q + i] * J[i][jj];
      mu[c * Q + jj] = s;
    }
    if (!(flags && (flags[c] & FLAG_NOFORCE)))
      for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += lam[c * Q + i] * JF[i][d];
        dF[c * 3 + d] = s;
      }
  }
  double acc[3] = {0, 0, 0};
  for (long c = 0; c < g->n; ++c)
    for (int d = 0; d < 3; ++d) acc[d] += dF[c * 3 + d];
  for (int d = 0; d < 3; ++d) dLdF[d] += acc[d];
  free(dF);
  return 0;
}

/* The transpose of stream_push (internal layout), as a gather:
 * lam_i(y) = mu_i(y + c_i) if that cell is fluid, else mu_{opp i}(y); 0 on
 * solid cells.  The moving-wall correction is a constant of the streaming
 * and has no transpose. */
static void stream_transpose_aos(const grid *g, const uint8_t *flags, const double *mu,
                                 double *lam) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->nz; ++z)
    for (int y = 0; y < g->ny; ++y)
      for (int x = 0; x < g->nx; ++x) {
        long c = cell(g, x, y, z);
        for (int i = 0; i < Q; ++i) {
          double v = 0.0;
          if (!is_solid(flags, c)) {
            long t = cell(g, wrap(x + C[i][0], g->nx), wrap(y + C[i][1], g->ny),
                          wrap(z + C[i][2], g->nz));
            v = !is_solid(flags, t) ? mu[t * Q + i] : mu[c * Q + OPP[i]];
          }
          lam[c * Q + i] = v;
        }
      }
}

/* One reverse step n+1 -> n.  Given f*(n) and lambda^{n+1}:
 *   f(n+1) = stream(f*(n));  mu = J(f(n+1))^T lambda^{n+1} at fluid cells;
 *   dLdF += JF(f(n+1))^T lambda^{n+1} at forced fluid cells;
 *   lambda^n = stream^T(mu).  The moving-wall correction is a constant of
 *   the streaming, so it enters f(n+1) but not the transpose. */
int oracle_adjoint_step(int nx, int ny, int nz, double tau, const double *F,
                        const uint8_t *flags, const double *wall_u, int incomp,
                        const double *fn_abi,
                        const double *lam_np1_abi, double *lam_n_abi,
                        double *dLdF) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *a = malloc((size_t)g.n * Q * sizeof(double));
  double *b = calloc((size_t)g.n * Q, sizeof(double));
  double *lam = malloc((size_t)g.n * Q * sizeof(double));
  double *mu = calloc((size_t)g.n * Q, sizeof(double));
  int rc = (a && b && lam && mu) ? 0 : -2;
  if (!rc) {
    load_abi(&g, fn_abi, a);
    load_abi(&g, lam_np1_abi, lam);
    stream_push(&g, flags, wall_u, a, b);
    rc = adjoint_collide_aos(&g, 1.0 / tau, F, flags, incomp, b, lam, mu, dLdF);
  }
  if (!rc) {
    stream_transpose_aos(&g, flags, mu, a);
    store_abi(&g, a, lam_n_abi);
  }
  free(a);
  free(b);
  free(lam);
  free(mu);
  return rc;
}

/* The collision's part of the reverse step on its own (interface layout):
 * mu = J(f_pre)^T lambda and dLdF += JF(f_pre)^T lambda at a given
 * pre-collision state f_pre. */
int oracle_adjoint_collide(int nx, int ny, int nz, double tau, const double *F,
                           const uint8_t *flags, int incomp, const double *fpre_abi,
                           const double *lam_abi, double *mu_abi, double *dLdF) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *f = malloc((size_t)g.n * Q * sizeof(double));
  double *lam = malloc((size_t)g.n * Q * sizeof(double));
  double *mu = malloc((size_t)g.n * Q * sizeof(double));
  int rc = (f && lam && mu) ? 0 : -2;
  if (!rc) {
    load_abi(&g, fpre_abi, f);
    load_abi(&g, lam_abi, lam);
    rc = adjoint_collide_aos(&g, 1.0 / tau, F, flags, incomp, f, lam, mu, dLdF);
  }
  if (!rc) store_abi(&g, mu, mu_abi);
  free(f);
  free(lam);
  free(mu);
  return rc;
}

/* The streaming's part on its own (interface layout): lambda = stream^T(mu),
 * the transposed streaming with half-way bounce-back. */
int oracle_stream_transpose(int nx, int ny, int nz, const uint8_t *flags,
                            const double *mu_abi, double *lam_abi) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
  double *mu = malloc((size_t)g.n * Q * sizeof(double));
  double *lam = malloc((size_t)g.n * Q * sizeof(double));
  if (!mu || !lam) {
    free(mu);
    free(lam);
    return -2;
  }
  load_abi(&g, mu_abi, mu);
  stream_transpose_aos(&g, flags, mu, lam);
  store_abi(&g, lam, lam_abi);
  free(mu);
  free(lam);
  return 0;
}

/* Initial-state adjoint: f*(0)_i = f^eq_i(rho0, u0) on fluid cells, so
 *   dL/du0 = sum_i lambda^0_i d f^eq_i / d u,  dL/drho0 = sum_i lambda^0_i d f^eq_i / d rho.
 * rho0 may be NULL (uniform 1); dL_drho0 may be NULL. */
int oracle_adjoint_init(int nx, int ny, int nz, const uint8_t *flags, int incomp,
                        const double *rho0, const double *u0,
                        const double *lam0_abi, double *dL_du0,
                        double *dL_drho0) {
  if (lattice_init() || check_dims(nx, ny, nz)) return -1;
  grid g = {nx, ny, nz, (long)nx * ny * nz};
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g.n; ++c) {
    double gu[3] = {0, 0, 0}, gr = 0.0;
    if (!is_solid(flags, c)) {
      double rho = rho0 ? rho0[c] : 1.0;
      double u[3] = {0, 0, 0};
      if (u0)
        for (int d = 0; d < 3; ++d) u[d] = u0[(long)d * g.n + c];
      double uu = dot3(u, u);
      for (int k = 0; k < Q; ++k) {
        int i = ABI2INT[k];
        double lam = lam0_abi[(long)k * g.n + c];
        double cu = cdot(i, u);
        double rho_u = incomp ? 1.0 : rho;
        gr += lam * (incomp ? W[i] : W[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        for (int a = 0; a < 3; ++a)
          gu[a] += lam * W[i] * rho_u * (3.0 * C[i][a] + 9.0 * cu * C[i][a] - 3.0 * u[a]);
      }
    }
    for (int a = 0; a < 3; ++a) dL_du0[(long)a * g.n + c] = gu[a];
    if (dL_drho0) dL_drho0[c] = gr;
  }
  return 0;
}

/* Host copy probe (STREAM copy c = a of the paper's Sec. 3 case study), to
 * state the host's attainable bandwidth next to the oracle timing. */
double oracle_host_copy(double *c, const double *a, long n, int reps) {
  for (int r = 0; r < reps; ++r) {
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) c[k] = a[k];
  }
  return c[n - 1];
}

int oracle_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of the following oracle calls (for the CPU timing). */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#endif
  return oracle_threads();
}
