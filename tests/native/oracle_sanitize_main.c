/* Driver of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (a CPU build; test infrastructure).  Exercises every exported function of
 * oracle/lbmref.c on small lattices -- ragged shapes, every boundary kind, a
 * moving wall, a per-node force field, sampled single-node steps -- so that
 * an out-of-bounds index or undefined arithmetic in the oracle aborts the
 * run.  Prints one line per case and "sanitize: ok" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t nx, ny;
  double omega[9];
  double fx, fy;
  const double* force;
  int32_t bc[4];
  double wall_u[4];
  double rho0;
} lbmref_params;

void lbmref_source(double Fx, double Fy, double ux, double uy, double S[9]);
void lbmref_collide(const double om[9], double Fx, double Fy, const double fb[9], double out[9]);
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9]);
void lbmref_kmatrix(double out[81]);
void lbmref_init(const lbmref_params* p, const double* rho, const double* ux, const double* uy, double* f);
void lbmref_step(const lbmref_params* p, double* f, double* tmp, int64_t nsteps);
void lbmref_step_at(const lbmref_params* p, const double* f, int64_t count, const int32_t* xs,
                    const int32_t* ys, double* out);
void lbmref_macroscopic(const lbmref_params* p, const double* f, double* rho, double* ux, double* uy,
                        double* sxx, double* syy, double* sxy);
void lbmref_diagnostics(const lbmref_params* p, const double* f, double out[4]);

static double uniform(uint64_t* s) {  /* splitmix64, top 53 bits */
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) / 9007199254740992.0;
}

static int run_case(int nx, int ny, const int bc[4], const double wall_u[4], int with_force) {
  const size_t n = (size_t)nx * ny;
  double* rho = malloc(n * sizeof(double));
  double* ux = malloc(n * sizeof(double));
  double* uy = malloc(n * sizeof(double));
  double* frc = malloc(2 * n * sizeof(double));
  double* f = malloc(9 * n * sizeof(double));
  double* tmp = malloc(9 * n * sizeof(double));
  double* out[6];
  for (int k = 0; k < 6; ++k) out[k] = malloc(n * sizeof(double));
  uint64_t seed = (uint64_t)nx * 1000003u + (uint64_t)ny;
  for (size_t i = 0; i < n; ++i) {
    rho[i] = 1.0 + 0.01 * (uniform(&seed) - 0.5);
    ux[i] = 0.04 * (uniform(&seed) - 0.5);
    uy[i] = 0.04 * (uniform(&seed) - 0.5);
    frc[i] = 1e-4 * (uniform(&seed) - 0.5);
    frc[n + i] = 1e-4 * (uniform(&seed) - 0.5);
  }
  lbmref_params p;
  p.nx = nx;
  p.ny = ny;
  for (int k = 0; k < 9; ++k) p.omega[k] = 0.0;
  p.omega[3] = 1.1;
  p.omega[4] = p.omega[5] = 1.0 / 0.7;
  p.omega[6] = 0.9;
  p.omega[7] = 1.2;
  p.omega[8] = 1.3;
  p.fx = with_force ? 0.0 : 2e-6;
  p.fy = with_force ? 0.0 : -1e-6;
  p.force = with_force ? frc : NULL;
  for (int s = 0; s < 4; ++s) {
    p.bc[s] = bc[s];
    p.wall_u[s] = wall_u[s];
  }
  p.rho0 = 1.0;
  lbmref_init(&p, rho, ux, uy, f);
  lbmref_step(&p, f, tmp, 7);
  int32_t xs[4] = {0, nx - 1, nx / 2, 0}, ys[4] = {0, ny - 1, ny / 2, ny - 1};
  double at[4 * 9];
  lbmref_step_at(&p, f, 4, xs, ys, at);
  lbmref_macroscopic(&p, f, out[0], out[1], out[2], out[3], out[4], out[5]);
  double d[4];
  lbmref_diagnostics(&p, f, d);
  int bad = !(isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]) && isfinite(d[3]));
  for (int k = 0; k < 36; ++k) bad |= !isfinite(at[k]);
  printf("case %dx%d bc %d%d%d%d force %d: mass %.15g\n", nx, ny, bc[0], bc[1], bc[2], bc[3], with_force, d[0]);
  for (int k = 0; k < 6; ++k) free(out[k]);
  free(rho); free(ux); free(uy); free(frc); free(f); free(tmp);
  return bad;
}

int main(void) {
  double om[9] = {0, 0, 0, 1.0, 1.25, 1.25, 1.0, 1.0, 1.0}, fb[9], post[9], S[9], K[81];
  lbmref_equilibrium(1.0, 0.02, -0.01, fb);
  lbmref_collide(om, 1e-5, 2e-5, fb, post);
  lbmref_source(1e-5, 2e-5, 0.02, -0.01, S);
  lbmref_kmatrix(K);
  const int shapes[5][2] = {{2, 2}, {3, 7}, {17, 5}, {33, 31}, {64, 3}};
  const int bcs[3][4] = {{0, 0, 0, 0}, {0, 0, 1, 1}, {1, 1, 1, 1}};
  const double wu[3][4] = {{0, 0, 0, 0}, {0, 0, 0.02, 0.1}, {0.01, -0.02, 0.03, 0.1}};
  int bad = 0;
  for (int s = 0; s < 5; ++s)
    for (int b = 0; b < 3; ++b)
      for (int fo = 0; fo < 2; ++fo) bad |= run_case(shapes[s][0], shapes[s][1], bcs[b], wu[b], fo);
  if (bad) {
    printf("sanitize: non-finite result\n");
    return 1;
  }
  printf("sanitize: ok\n");
  return 0;
}
