/*
 * oracle/lbmref.c -- FP64 CPU oracle of the cascaded (central-moment MRT) D2Q9
 * lattice Boltzmann method with central-moment forcing, after Ning & Premnath,
 * "Numerical Study of the Properties of the Central Moment Lattice Boltzmann
 * Method", Section II (the cascaded LBM), plus the boundary treatments of
 * Section III (halfway bounce-back, moving-wall bounce-back).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU path.
 *
 * Every per-cell formula below is the paper's explicit one, written out in
 * its order and notation:
 *   - hydrodynamic fields            Sec. II, Eqs. for rho and rho*u_i
 *   - raw moments of f-bar           Sec. II, compact-summation equations
 *   - raw source moments sigma'      Sec. II, Eq. (S value)
 *   - source projections m^s         Sec. II, the m^s_0..m^s_8 list
 *   - source in velocity space S_a   Sec. II, the S_0..S_8 list
 *   - collision kernels g3..g8       Sec. II, Eqs. (collisionkernelg3-g8)
 *   - post-collision populations     Sec. II, the f~_0..f~_8 list
 *   - stream step                    Sec. II, Eq. (transformed f), 2nd line
 *   - strain rate                    Sec. II, Eqs. (strainrate1-3)
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   E3  g6 and g7 use the raw source moments sigma'_xxy, sigma'_xyy.  With the
 *       unprimed (central, identically zero) values the kernels do not relax
 *       each central moment at its own rate.
 *   E4  The strain-rate equations are combined from the three Chapman-Enskog
 *       relations for f3neq, f4neq, f5neq (valid for omega3 != omega4):
 *         dx jx = -3/4 (w3 f3neq + w4 f4neq), dy jy = -3/4 (w3 f3neq - w4 f4neq),
 *         dx jy + dy jx = -3 w5 f5neq; strain = those divided by rho.
 *   E6  Moving-wall term 6 rho0 w_a (e_a . U_wall), i.e. e_ax for a lid moving
 *       in x, with the reference density rho0.  A link that crosses two walls
 *       runs through the corner point where they meet; that point is taken
 *       at rest, so such a link is plain bounce-back with no wall term.  (With
 *       the lid term on these two links the cavity converges at first order
 *       only; without it, at the second order Sec. III.C reports.)
 *   Initial state: f-bar = f^eq - S/2, f^eq being the D2Q9 distribution whose
 *       central moments are the Maxwellian ones (Sec. II, kappa^eq list).
 *   Walls sit half a lattice spacing outside the first/last fluid node.
 *
 * Layout: populations f[a][y][x] (a = 0..8, row-major, no padding), FP64.
 * Direction order as in Sec. II:  e_x = (0,1,0,-1,0,1,-1,-1,1),
 *                                 e_y = (0,0,1,0,-1,1,1,-1,-1).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Lattice weights w_a used by the moving-wall correction (Sec. III, lid BC). */
static const double WGT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* The orthogonal moment matrix K exactly as printed in Sec. II (Eq. after
 * "K value"): row a = population a, column b = basis vector |K_b>. */
static const double KMAT[9][9] = {
    {1, 0, 0, -4, 0, 0, 0, 0, 4},    {1, 1, 0, -1, 1, 0, 0, 2, -2},
    {1, 0, 1, -1, -1, 0, 2, 0, -2},  {1, -1, 0, -1, 1, 0, 0, -2, -2},
    {1, 0, -1, -1, -1, 0, -2, 0, -2}, {1, 1, 1, 2, 0, 1, -1, -1, 1},
    {1, -1, 1, 2, 0, -1, -1, 1, 1},  {1, -1, -1, 2, 0, 1, 1, 1, 1},
    {1, 1, -1, 2, 0, -1, 1, -1, 1}};

typedef struct {
  int32_t nx, ny;
  double omega[9];     /* omega[3..8] used (omega[4] = omega[5] = 1/tau)     */
  double fx, fy;       /* uniform body force, used when force == NULL        */
  const double* force; /* per-node body force [2][ny][nx], or NULL           */
  int32_t bc[4];       /* x_lo, x_hi, y_lo, y_hi: 0 periodic, 1 wall          */
  double wall_u[4];    /* tangential wall velocity of each side              */
  double rho0;         /* reference density (moving-wall term)               */
} lbmref_params;

/* ---------------------------------------------------------------- per node */

/* Hydrodynamic fields from f-bar (Sec. II): rho = sum f-bar,
 * rho u_i = sum f-bar e_i + F_i / 2. */
static void fields(const double fb[9], double Fx, double Fy, double* rho,
                   double* ux, double* uy) {
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int a = 0; a < 9; ++a) {
    r += fb[a];
    jx += fb[a] * EX[a];
    jy += fb[a] * EY[a];
  }
  *rho = r;
  *ux = (jx + 0.5 * Fx) / r;
  *uy = (jy + 0.5 * Fy) / r;
}

/* Raw source moments sigma' (Sec. II, Eq. "S value"). Index order:
 * 0, x, y, xx, yy, xy, xxy, xyy, xxyy. */
static void source_raw_moments(double Fx, double Fy, double ux, double uy,
                               double sg[9]) {
  sg[0] = 0.0;
  sg[1] = Fx;
  sg[2] = Fy;
  sg[3] = 2.0 * Fx * ux;
  sg[4] = 2.0 * Fy * uy;
  sg[5] = Fx * uy + Fy * ux;
  sg[6] = Fy * ux * ux + 2.0 * Fx * ux * uy;
  sg[7] = Fx * uy * uy + 2.0 * Fy * uy * ux;
  sg[8] = 2.0 * Fx * ux * uy * uy + 2.0 * Fy * uy * ux * ux;
}

/* Source projections m^s_b = <K_b|S> (Sec. II, m^s_0..m^s_8). */
static void source_projections(double Fx, double Fy, double ux, double uy,
                               double ms[9]) {
  ms[0] = 0.0;
  ms[1] = Fx;
  ms[2] = Fy;
  ms[3] = 6.0 * (Fx * ux + Fy * uy);
  ms[4] = 2.0 * (Fx * ux - Fy * uy);
  ms[5] = Fx * uy + Fy * ux;
  ms[6] = (2.0 - 3.0 * ux * ux) * Fy - 6.0 * Fx * ux * uy;
  ms[7] = (2.0 - 3.0 * uy * uy) * Fx - 6.0 * Fy * uy * ux;
  ms[8] = 6.0 * ((3.0 * uy * uy - 2.0) * Fx * ux + (3.0 * ux * ux - 2.0) * Fy * uy);
}

/* Source in velocity space S_a (Sec. II, S_0..S_8, the exact inversion of
 * K^T S = m^s). */
void lbmref_source(double Fx, double Fy, double ux, double uy, double S[9]) {
  double m[9];
  source_projections(Fx, Fy, ux, uy, m);
  S[0] = (-m[3] + m[8]) / 9.0;
  S[1] = (6 * m[1] - m[3] + 9 * m[4] + 6 * m[7] - 2 * m[8]) / 36.0;
  S[2] = (6 * m[2] - m[3] - 9 * m[4] + 6 * m[6] - 2 * m[8]) / 36.0;
  S[3] = (-6 * m[1] - m[3] + 9 * m[4] - 6 * m[7] - 2 * m[8]) / 36.0;
  S[4] = (-6 * m[2] - m[3] - 9 * m[4] - 6 * m[6] - 2 * m[8]) / 36.0;
  S[5] = (6 * m[1] + 6 * m[2] + 2 * m[3] + 9 * m[5] - 3 * m[6] - 3 * m[7] + m[8]) / 36.0;
  S[6] = (-6 * m[1] + 6 * m[2] + 2 * m[3] - 9 * m[5] - 3 * m[6] + 3 * m[7] + m[8]) / 36.0;
  S[7] = (-6 * m[1] - 6 * m[2] + 2 * m[3] + 9 * m[5] + 3 * m[6] + 3 * m[7] + m[8]) / 36.0;
  S[8] = (6 * m[1] - 6 * m[2] + 2 * m[3] - 9 * m[5] + 3 * m[6] - 3 * m[7] + m[8]) / 36.0;
}

/* One cascaded collision of a node (Sec. II): f-bar -> f~-bar = f-bar +
 * (K g)_a + S_a.  om[3..8] are the relaxation rates omega_3..omega_8. */
void lbmref_collide(const double om[9], double Fx, double Fy,
                    const double fb[9], double out[9]) {
  double rho, ux, uy;
  fields(fb, Fx, Fy, &rho, &ux, &uy);

  /* Raw moments of f-bar via the compact summation operator (Sec. II). */
  const double kxx = fb[1] + fb[3] + fb[5] + fb[6] + fb[7] + fb[8];
  const double kyy = fb[2] + fb[4] + fb[5] + fb[6] + fb[7] + fb[8];
  const double kxy = (fb[5] + fb[7]) - (fb[6] + fb[8]);
  const double kxxy = (fb[5] + fb[6]) - (fb[7] + fb[8]);
  const double kxyy = (fb[5] + fb[8]) - (fb[6] + fb[7]);
  const double kxxyy = fb[5] + fb[6] + fb[7] + fb[8];

  double sg[9];
  source_raw_moments(Fx, Fy, ux, uy, sg);
  const double sxx = sg[3], syy = sg[4], sxy = sg[5], sxxy = sg[6],
               sxyy = sg[7], sxxyy = sg[8];

  const double ux2 = ux * ux, uy2 = uy * uy;

  /* Collision kernels g3..g8 (Sec. II, Eqs. collisionkernelg3-g8; reading
   * E3: sigma' in g6 and g7). */
  const double g3 = om[3] / 12.0 *
                    (2.0 / 3.0 * rho + rho * (ux2 + uy2) - (kxx + kyy) -
                     0.5 * (sxx + syy));
  const double g4 = om[4] / 4.0 *
                    (rho * (ux2 - uy2) - (kxx - kyy) - 0.5 * (sxx - syy));
  const double g5 = om[5] / 4.0 * (rho * ux * uy - kxy - 0.5 * sxy);
  const double g6 = om[6] / 4.0 *
                        (2.0 * rho * ux2 * uy + kxxy - 2.0 * ux * kxy -
                         uy * kxx - 0.5 * sxxy) -
                    0.5 * uy * (3.0 * g3 + g4) - 2.0 * ux * g5;
  const double g7 = om[7] / 4.0 *
                        (2.0 * rho * ux * uy2 + kxyy - 2.0 * uy * kxy -
                         ux * kyy - 0.5 * sxyy) -
                    0.5 * ux * (3.0 * g3 - g4) - 2.0 * uy * g5;
  const double g8 =
      om[8] / 4.0 *
          (1.0 / 9.0 * rho + 3.0 * rho * ux2 * uy2 -
           (kxxyy - 2.0 * ux * kxyy - 2.0 * uy * kxxy + ux2 * kyy + uy2 * kxx +
            4.0 * ux * uy * kxy) -
           0.5 * sxxyy) -
      2.0 * g3 - 0.5 * uy2 * (3.0 * g3 + g4) - 0.5 * ux2 * (3.0 * g3 - g4) -
      4.0 * ux * uy * g5 - 2.0 * uy * g6 - 2.0 * ux * g7;

  /* Conserved kernels vanish: g0 = g1 = g2 = 0. */
  double S[9];
  lbmref_source(Fx, Fy, ux, uy, S);

  /* Post-collision populations (Sec. II, f~_0..f~_8). */
  out[0] = fb[0] + (-4.0 * (g3 - g8)) + S[0];
  out[1] = fb[1] + (-g3 + g4 + 2.0 * (g7 - g8)) + S[1];
  out[2] = fb[2] + (-g3 - g4 + 2.0 * (g6 - g8)) + S[2];
  out[3] = fb[3] + (-g3 + g4 - 2.0 * (g7 + g8)) + S[3];
  out[4] = fb[4] + (-g3 - g4 - 2.0 * (g6 + g8)) + S[4];
  out[5] = fb[5] + (2.0 * g3 + g5 - g6 - g7 + g8) + S[5];
  out[6] = fb[6] + (2.0 * g3 - g5 - g6 + g7 + g8) + S[6];
  out[7] = fb[7] + (2.0 * g3 + g5 + g6 + g7 + g8) + S[7];
  out[8] = fb[8] + (2.0 * g3 - g5 + g6 - g7 + g8) + S[8];
}

/* Binomial coefficient for m <= 2. */
static double binom(int p, int q) { return (p == 2 && q == 1) ? 2.0 : 1.0; }

/* Distribution with prescribed central moments about u (Sec. II): the raw
 * moments follow from the binomial formula with +u (the inverse of the
 * central-moment shift), the orthogonal projections <K_b|f> are the
 * combinations of monomials that define |K_b>, and f = K D^-1 (K^T f) with
 * D = diag(<K_b|K_b>) (orthogonality of K).  cm order: 0, x, y, xx, yy, xy,
 * xxy, xyy, xxyy. */
static void from_central_moments(const double cm[9], double ux, double uy,
                                 double f[9]) {
  /* c[m][n] = central moment of order (m, n). */
  double c[3][3];
  c[0][0] = cm[0]; c[1][0] = cm[1]; c[0][1] = cm[2];
  c[2][0] = cm[3]; c[0][2] = cm[4]; c[1][1] = cm[5];
  c[2][1] = cm[6]; c[1][2] = cm[7]; c[2][2] = cm[8];
  double M[3][3];
  double upx[3] = {1.0, ux, ux * ux}, upy[3] = {1.0, uy, uy * uy};
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 3; ++n) {
      double s = 0.0;
      for (int i = 0; i <= m; ++i)
        for (int j = 0; j <= n; ++j)
          s += binom(m, i) * binom(n, j) * upx[m - i] * upy[n - j] * c[i][j];
      M[m][n] = s;
    }
  /* <K_b|f> from the monomial definitions of |K_b> (Sec. II, Eq. K value). */
  double mk[9];
  mk[0] = M[0][0];
  mk[1] = M[1][0];
  mk[2] = M[0][1];
  mk[3] = 3.0 * (M[2][0] + M[0][2]) - 4.0 * M[0][0];
  mk[4] = M[2][0] - M[0][2];
  mk[5] = M[1][1];
  mk[6] = -3.0 * M[2][1] + 2.0 * M[0][1];
  mk[7] = -3.0 * M[1][2] + 2.0 * M[1][0];
  mk[8] = 9.0 * M[2][2] - 6.0 * (M[2][0] + M[0][2]) + 4.0 * M[0][0];
  double D[9];
  for (int b = 0; b < 9; ++b) {
    D[b] = 0.0;
    for (int a = 0; a < 9; ++a) D[b] += KMAT[a][b] * KMAT[a][b];
  }
  for (int a = 0; a < 9; ++a) {
    double s = 0.0;
    for (int b = 0; b < 9; ++b) s += KMAT[a][b] * mk[b] / D[b];
    f[a] = s;
  }
}

/* Discrete equilibrium: central moments equal the Maxwellian ones
 * (rho, 0, 0, rho/3, rho/3, 0, 0, 0, rho/9), Sec. II kappa^eq list. */
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9]) {
  const double cs2 = 1.0 / 3.0;
  const double cm[9] = {rho, 0.0, 0.0, cs2 * rho, cs2 * rho,
                        0.0, 0.0, 0.0, cs2 * cs2 * rho};
  from_central_moments(cm, ux, uy, feq);
}

/* Expose the printed K matrix (for the test that it is transcribed right). */
void lbmref_kmatrix(double out[81]) {
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) out[a * 9 + b] = KMAT[a][b];
}

/* -------------------------------------------------------------- lattice */

static inline size_t idx(const lbmref_params* p, int a, int y, int x) {
  return ((size_t)a * p->ny + y) * p->nx + x;
}

static inline void node_force(const lbmref_params* p, int y, int x, double* Fx,
                              double* Fy) {
  if (p->force) {
    const size_t n = (size_t)p->nx * p->ny;
    *Fx = p->force[(size_t)y * p->nx + x];
    *Fy = p->force[n + (size_t)y * p->nx + x];
  } else {
    *Fx = p->fx;
    *Fy = p->fy;
  }
}

/* Initial state f-bar = f^eq(rho, u) - S(u, F)/2 (transformed variable,
 * Sec. II) from node fields rho, ux, uy, each [ny][nx]. */
void lbmref_init(const lbmref_params* p, const double* rho, const double* ux,
                 const double* uy, double* f) {
#pragma omp parallel for schedule(static) if ((int64_t)p->nx * p->ny >= 16384)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const size_t c = (size_t)y * p->nx + x;
      double Fx, Fy, feq[9], S[9];
      node_force(p, y, x, &Fx, &Fy);
      lbmref_equilibrium(rho[c], ux[c], uy[c], feq);
      lbmref_source(Fx, Fy, ux[c], uy[c], S);
      for (int a = 0; a < 9; ++a) f[idx(p, a, y, x)] = feq[a] - 0.5 * S[a];
    }
}

/* Collide every node: post = f~-bar(f-bar). */
static void collide_all(const lbmref_params* p, const double* f, double* post) {
#pragma omp parallel for schedule(static) if ((int64_t)p->nx * p->ny >= 16384)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double fb[9], out[9], Fx, Fy;
      for (int a = 0; a < 9; ++a) fb[a] = f[idx(p, a, y, x)];
      node_force(p, y, x, &Fx, &Fy);
      lbmref_collide(p->omega, Fx, Fy, fb, out);
      for (int a = 0; a < 9; ++a) post[idx(p, a, y, x)] = out[a];
    }
}

/* Value that arrives at node (x, y) along direction a after streaming the
 * post-collision field `post` (Sec. II, 2nd line of Eq. transformed f):
 * f-bar_a(x) = f~-bar_a(x - e_a).  If x - e_a lies beyond a wall (halfway
 * bounce-back, Sec. III Poiseuille), the population that left x towards that
 * wall returns reversed: f-bar_a(x) = f~-bar_opp(a)(x), plus the moving-wall
 * term 6 rho0 w_a (e_a . U_wall) if exactly one wall is crossed (Sec. III
 * cavity, reading E6: a link crossing two walls meets their corner point,
 * which is at rest).  Periodic sides wrap. */
static double pulled(const lbmref_params* p, const double* post, int a, int y,
                     int x) {
  int sx = x - EX[a], sy = y - EY[a];
  int hit_xlo = 0, hit_xhi = 0, hit_ylo = 0, hit_yhi = 0;
  if (sx < 0) { if (p->bc[0]) hit_xlo = 1; else sx += p->nx; }
  if (sx >= p->nx) { if (p->bc[1]) hit_xhi = 1; else sx -= p->nx; }
  if (sy < 0) { if (p->bc[2]) hit_ylo = 1; else sy += p->ny; }
  if (sy >= p->ny) { if (p->bc[3]) hit_yhi = 1; else sy -= p->ny; }
  const int crossed = hit_xlo + hit_xhi + hit_ylo + hit_yhi;
  if (crossed) {
    const double k = 6.0 * p->rho0 * WGT[a];
    double wterm = 0.0;
    /* x walls move tangentially in y; y walls move tangentially in x. */
    if (crossed == 1) {
      if (hit_xlo) wterm = k * EY[a] * p->wall_u[0];
      if (hit_xhi) wterm = k * EY[a] * p->wall_u[1];
      if (hit_ylo) wterm = k * EX[a] * p->wall_u[2];
      if (hit_yhi) wterm = k * EX[a] * p->wall_u[3];
    }
    return post[idx(p, OPP[a], y, x)] + wterm;
  }
  return post[idx(p, a, sy, sx)];
}

static void stream_all(const lbmref_params* p, const double* post, double* f) {
#pragma omp parallel for schedule(static) if ((int64_t)p->nx * p->ny >= 16384)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x)
      for (int a = 0; a < 9; ++a) f[idx(p, a, y, x)] = pulled(p, post, a, y, x);
}

/* Advance the pre-collision state f (f-bar at time n) by nsteps full
 * collide-and-stream steps, in place.  `tmp` has the size of f. */
void lbmref_step(const lbmref_params* p, double* f, double* tmp,
                 int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s) {
    collide_all(p, f, tmp);
    stream_all(p, tmp, f);
  }
}

/* One step evaluated only at the listed nodes: out[k][a] is f-bar_a at node
 * (xs[k], ys[k]) at time n+1, computed from the full pre-collision field f
 * at time n (collide the source node, then stream). */
void lbmref_step_at(const lbmref_params* p, const double* f, int64_t count,
                    const int32_t* xs, const int32_t* ys, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    const int x = xs[k], y = ys[k];
    for (int a = 0; a < 9; ++a) {
      int sx = x - EX[a], sy = y - EY[a];
      int wall = 0;
      double wterm = 0.0;
      const double kw = 6.0 * p->rho0 * WGT[a];
      if (sx < 0) { if (p->bc[0]) { ++wall; wterm = kw * EY[a] * p->wall_u[0]; } else sx += p->nx; }
      if (sx >= p->nx) { if (p->bc[1]) { ++wall; wterm = kw * EY[a] * p->wall_u[1]; } else sx -= p->nx; }
      if (sy < 0) { if (p->bc[2]) { ++wall; wterm = kw * EX[a] * p->wall_u[2]; } else sy += p->ny; }
      if (sy >= p->ny) { if (p->bc[3]) { ++wall; wterm = kw * EX[a] * p->wall_u[3]; } else sy -= p->ny; }
      if (wall > 1) wterm = 0.0; /* corner point: at rest (reading E6) */
      const int cx = wall ? x : sx, cy = wall ? y : sy;
      const int ca = wall ? OPP[a] : a;
      double fb[9], post[9], Fx, Fy;
      for (int b = 0; b < 9; ++b) fb[b] = f[idx(p, b, cy, cx)];
      node_force(p, cy, cx, &Fx, &Fy);
      lbmref_collide(p->omega, Fx, Fy, fb, post);
      out[k * 9 + a] = post[ca] + wterm;
    }
  }
}

/* Density, velocity and strain rate at every node from the pre-collision
 * state (Sec. II hydrodynamic fields; strain rate by reading E4).  Any output
 * pointer may be NULL. */
void lbmref_macroscopic(const lbmref_params* p, const double* f, double* rho,
                        double* ux, double* uy, double* sxx, double* syy,
                        double* sxy) {
  const double* om = p->omega;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const size_t c = (size_t)y * p->nx + x;
      double fb[9], Fx, Fy, r, vx, vy, S[9];
      for (int a = 0; a < 9; ++a) fb[a] = f[idx(p, a, y, x)];
      node_force(p, y, x, &Fx, &Fy);
      fields(fb, Fx, Fy, &r, &vx, &vy);
      if (rho) rho[c] = r;
      if (ux) ux[c] = vx;
      if (uy) uy[c] = vy;
      if (sxx || syy || sxy) {
        /* Non-equilibrium raw moments of f = f-bar + S/2 (Sec. II). */
        lbmref_source(Fx, Fy, vx, vy, S);
        double kxx = 0.0, kyy = 0.0, kxy = 0.0;
        for (int a = 0; a < 9; ++a) {
          const double fa = fb[a] + 0.5 * S[a];
          kxx += fa * EX[a] * EX[a];
          kyy += fa * EY[a] * EY[a];
          kxy += fa * EX[a] * EY[a];
        }
        const double f3neq = (kxx + kyy) - (2.0 / 3.0 * r + r * (vx * vx + vy * vy));
        const double f4neq = (kxx - kyy) - r * (vx * vx - vy * vy);
        const double f5neq = kxy - r * vx * vy;
        const double dxjx = -0.75 * (om[3] * f3neq + om[4] * f4neq);
        const double dyjy = -0.75 * (om[3] * f3neq - om[4] * f4neq);
        const double shear = -3.0 * om[5] * f5neq;
        if (sxx) sxx[c] = dxjx / r;
        if (syy) syy[c] = dyjy / r;
        if (sxy) sxy[c] = 0.5 * shear / r;
      }
    }
}

/* Global sums: out = {sum rho, sum rho ux, sum rho uy, 1/2 sum rho |u|^2}. */
void lbmref_diagnostics(const lbmref_params* p, const double* f, double out[4]) {
  double m = 0.0, px = 0.0, py = 0.0, e = 0.0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double fb[9], Fx, Fy, r, vx, vy;
      for (int a = 0; a < 9; ++a) fb[a] = f[idx(p, a, y, x)];
      node_force(p, y, x, &Fx, &Fy);
      fields(fb, Fx, Fy, &r, &vx, &vy);
      m += r;
      px += r * vx;
      py += r * vy;
      e += 0.5 * r * (vx * vx + vy * vy);
    }
  out[0] = m;
  out[1] = px;
  out[2] = py;
  out[3] = e;
}

int lbmref_num_threads(void);
#ifdef _OPENMP
#include <omp.h>
int lbmref_num_threads(void) { return omp_get_max_threads(); }
#else
int lbmref_num_threads(void) { return 1; }
#endif
