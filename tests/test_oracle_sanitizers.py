"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

A small C driver, compiled together with oracle/mcc_oracle.c by gcc with
-fsanitize=address,undefined (errors abort), steps a ragged population
(empty, single-particle, odd and larger cells; three species; lognormal
weights) through every entry point the tests use: the sorted step in each
method, pairing, precision option and failure policy, the relativistic step,
hard spheres, the unsorted step and the binning, with two OpenMP threads.
The run must end cleanly: no out-of-bounds access, use after free, leak,
signed overflow or other undefined behaviour in the oracle's C.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mcc_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_collide_sorted(int64_t n, int32_t n_cells, int32_t n_species, const int64_t *offsets,
    const double *mass, const double *charge, int32_t n_coll, const int32_t *coll_a,
    const int32_t *coll_b, const double *w, double *vx, double *vy, double *vz,
    const double *cell_volume, double cell_volume_scalar, double dt, double coulomb_log,
    uint64_t seed, uint64_t step, int32_t method, int32_t pairing, int32_t relativistic,
    int32_t moment_correction, int32_t sort_by_weight, int32_t max_passes, int32_t keep_on_fail,
    double f_E, double eps0, double c, const int32_t *cell_list, int32_t n_list,
    int64_t *counters, double *diag, int32_t *cell_corr_pairs, const double *cross_section,
    int32_t uniform23);
int oracle_collide(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
    int32_t n_species, const double *mass, const double *charge, int32_t n_coll,
    const int32_t *coll_a, const int32_t *coll_b, const double *w, double *vx, double *vy,
    double *vz, const double *cell_volume, double cell_volume_scalar, double dt,
    double coulomb_log, uint64_t seed, uint64_t step, int32_t method, int32_t pairing,
    int32_t relativistic, int32_t moment_correction, int32_t sort_by_weight, int32_t max_passes,
    int32_t keep_on_fail, double f_E, double eps0, double c, int64_t *counters, double *diag,
    int32_t *cell_corr_pairs, const double *cross_section, int32_t uniform23);
int oracle_bin(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
    int32_t n_species, int64_t *offsets, int64_t *perm);
void oracle_set_threads(int32_t n);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static double uni(void) {  /* xorshift64*: test data only */
  st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
  return ((st * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0) + 1e-300;
}
static double gauss(void) { return sqrt(-2.0 * log(uni())) * cos(6.283185307179586 * uni()); }

int main(void) {
  enum { NC = 7, S = 3 };
  const int counts[NC][S] = {{0, 0, 0}, {1, 0, 2}, {5, 4, 3}, {17, 2, 9}, {64, 63, 1},
                             {0, 40, 33}, {150, 97, 120}};
  int64_t off[NC * S + 1];
  off[0] = 0;
  for (int k = 0; k < NC * S; ++k) off[k + 1] = off[k] + counts[k / S][k % S];
  const int64_t n = off[NC * S];
  double *w = malloc(sizeof(double) * n), *v0 = malloc(sizeof(double) * 3 * n);
  double *vx = malloc(sizeof(double) * n), *vy = malloc(sizeof(double) * n),
         *vz = malloc(sizeof(double) * n);
  int32_t *cells = malloc(sizeof(int32_t) * n), *spec = malloc(sizeof(int32_t) * n);
  for (int k = 0; k < NC * S; ++k)
    for (int64_t i = off[k]; i < off[k + 1]; ++i) {
      cells[i] = k / S;
      spec[i] = k % S;
      w[i] = exp(gauss());
      for (int d = 0; d < 3; ++d) v0[3 * i + d] = 0.3 * gauss() / (1.0 + k % S);
    }
  const double mass[S] = {1.0, 4.0, 50.0}, charge[S] = {-1.0, 2.0, 3.0};
  const int32_t ca[6] = {0, 1, 0, 2, 1, 0}, cb[6] = {0, 1, 1, 2, 2, 2};
  const double xs[6] = {0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
  int64_t counters[4];
  double diag[2];
  int32_t ccp[NC];
  int fails = 0;
  /* method, pairing, relativistic, correction, sort, passes, keep, uniform23 */
  const int cases[][8] = {{1, 0, 0, 1, 1, 1, 0, 0}, {0, 0, 0, 1, 1, 1, 0, 0}, {1, 0, 0, 1, 0, 3, 1, 0},
                          {1, 0, 0, 0, 1, 1, 0, 0}, {1, 0, 0, 1, 1, 1, 0, 1}, {1, 1, 0, 1, 1, 1, 0, 0},
                          {1, 2, 0, 1, 1, 1, 0, 0}, {1, 0, 1, 1, 1, 1, 0, 0}, {2, 0, 0, 1, 1, 2, 0, 0},
                          {2, 1, 0, 1, 1, 1, 1, 0}};
  const int ncase = (int)(sizeof(cases) / sizeof(cases[0]));
  oracle_set_threads(2);
  for (int c = 0; c < ncase; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = v0[3 * i];
      vy[i] = v0[3 * i + 1];
      vz[i] = v0[3 * i + 2];
    }
    const int rel = cases[c][2];
    for (int step = 0; step < 3; ++step) {
      const int rc = oracle_collide_sorted(n, NC, S, off, mass, charge, 6, ca, cb, w, vx, vy, vz,
          NULL, 1.0, 0.05, 10.0, 77, step, cases[c][0], cases[c][1], rel, cases[c][3],
          cases[c][4], cases[c][5], cases[c][6], 0.05, 1.0, rel ? 1.0 : INFINITY, NULL, 0,
          counters, diag, ccp, cases[c][0] == 2 ? xs : NULL, cases[c][7]);
      if (rc) {
        fprintf(stderr, "case %d step %d: rc %d\n", c, step, rc);
        ++fails;
      }
    }
  }
  /* the unsorted entry on a reversed order, and the binning */
  int32_t *rc_cells = malloc(sizeof(int32_t) * n), *rc_spec = malloc(sizeof(int32_t) * n);
  double *rw = malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) {
    rc_cells[i] = cells[n - 1 - i];
    rc_spec[i] = spec[n - 1 - i];
    rw[i] = w[n - 1 - i];
    vx[i] = v0[3 * (n - 1 - i)];
    vy[i] = v0[3 * (n - 1 - i) + 1];
    vz[i] = v0[3 * (n - 1 - i) + 2];
  }
  if (oracle_collide(n, rc_cells, rc_spec, NC, S, mass, charge, 6, ca, cb, rw, vx, vy, vz, NULL,
                     1.0, 0.05, 10.0, 77, 5, 1, 0, 0, 1, 1, 1, 0, 0.05, 1.0, INFINITY, counters,
                     diag, ccp, NULL, 0))
    ++fails;
  int64_t boff[NC * S + 1], *perm = malloc(sizeof(int64_t) * n);
  if (oracle_bin(n, rc_cells, rc_spec, NC, S, boff, perm)) ++fails;
  for (int k = 0; k <= NC * S; ++k)
    if (boff[k] != off[k]) ++fails;
  free(w); free(v0); free(vx); free(vy); free(vz); free(cells); free(spec);
  free(rc_cells); free(rc_spec); free(rw); free(perm);
  printf("sanitized oracle: %d cases, %d failures\n", ncase, fails);
  return fails ? 1 : 0;
}
"""


def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "driver.c")
        open(drv, "w").write(DRIVER)
        exe = os.path.join(d, "oracle_sanitized")
        flags = ["-std=gnu11", "-O1", "-g", "-ffp-contract=off", "-fopenmp",
                 "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"]
        r = subprocess.run([gcc, *flags, SRC, drv, "-o", exe, "-lm"], capture_output=True,
                           text=True)
        if r.returncode != 0 and "sanitize" in r.stderr:
            pytest.skip("gcc here has no sanitizer runtime: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
        assert "0 failures" in r.stdout
