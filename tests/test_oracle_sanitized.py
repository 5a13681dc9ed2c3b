"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc) and driven through a bulk run, a gated device run with
contact refill and window observables, and its single-event hooks: any
out-of-bounds access, use after free or undefined operation aborts the
driver."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
typedef struct {
  double m_eff[3], alpha[3], E_c[3]; int Z[3];
  double eps_s, eps_inf, rho, D_ac_eV, D_iv_eVm, hw_lo_eV, hw_iv_eV, u_ac;
  int mode, pad0; uint64_t seed; uint32_t instance; int n_particles, capacity;
  double dt_fs; int substeps, n_bins; double dE_eV, T0_K, T_init_K, N_D_m3;
  double F_bulk[3], L_nm[3]; int n_cells[3], pad1; double gate_x_nm[2], Vgs, Vds, phi_offset;
} cfg_t;
typedef struct { int intervals, pad; double rest[40]; } obs_t;
void *or_create(const cfg_t *, const double *);
void or_destroy(void *);
int or_run(void *, int, int);
void or_reset_window(void *);
void or_observables(const void *, void *);
void or_power_maps(const void *, double *, double *, double *);
int or_ncell(const void *);
void or_sample_selection(const void *, int, double, int, uint32_t, int, uint64_t *);
int or_steady_test(const double *, int, double *);
static cfg_t base(int mode) {
  cfg_t c; memset(&c, 0, sizeof c);
  double m[3] = {0.21, 0.25, 0.40}, a[3] = {0.19, 0.1, 0.0}, e[3] = {0.0, 1.95, 2.1};
  for (int v = 0; v < 3; ++v) { c.m_eff[v] = m[v]; c.alpha[v] = a[v]; c.E_c[v] = e[v]; }
  c.Z[0] = 1; c.Z[1] = 6; c.Z[2] = 1;
  c.eps_s = 8.9; c.eps_inf = 5.35; c.rho = 6095.0; c.D_ac_eV = 8.3; c.D_iv_eVm = 1e11;
  c.hw_lo_eV = 0.0912; c.hw_iv_eV = 0.0912; c.u_ac = 3338.0;
  c.mode = mode; c.seed = 1707; c.dt_fs = 1.0; c.n_bins = 3000; c.dE_eV = 1e-3;
  c.T0_K = 300.0; c.T_init_K = 300.0;
  return c;
}
int main(void) {
  cfg_t b = base(0);
  b.n_particles = b.capacity = 300; b.substeps = 10; b.N_D_m3 = 1e23; b.F_bulk[2] = 5e-2;
  void *o = or_create(&b, NULL);
  if (or_run(o, 20, 1) != 0) return 2;
  obs_t ob; or_observables(o, &ob);
  uint64_t cnt[11] = {0};
  or_sample_selection(o, 0, 0.5, 0, 7, 1000, cnt);
  or_destroy(o);
  cfg_t d = base(1);
  d.n_particles = 2000; d.capacity = 2600; d.substeps = 10; d.N_D_m3 = 1e24;
  d.L_nm[0] = 200.0; d.L_nm[1] = 60.0; d.L_nm[2] = 120.0;
  d.n_cells[0] = 20; d.n_cells[1] = 3; d.n_cells[2] = 6;
  d.gate_x_nm[0] = 50.0; d.gate_x_nm[1] = 150.0; d.Vgs = -0.5; d.Vds = 2.0;
  double *T = malloc(sizeof(double) * 360);
  for (int i = 0; i < 360; ++i) T[i] = 300.0 + 0.2 * i;
  o = or_create(&d, T);
  if (or_run(o, 10, 1) != 0) return 3;
  or_reset_window(o);
  if (or_run(o, 25, 1) != 0) return 4;
  or_observables(o, &ob);
  double *q = malloc(sizeof(double) * 3 * 360);
  or_power_maps(o, q, q + 360, q + 720);
  double s[41], out[4];
  for (int i = 0; i < 41; ++i) s[i] = i % 3;
  int f = or_steady_test(s, 41, out);
  printf("ok %d %d %g\n", ob.intervals, f, q[0]);
  free(q); free(T);
  or_destroy(o);
  return 0;
}
"""


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "drv.c")
        exe = os.path.join(d, "drv")
        open(drv, "w").write(DRIVER)
        flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
        try:
            subprocess.check_call(["gcc", "-std=c11", "-fopenmp", *flags, "-o", exe, drv,
                                   os.path.join(ROOT, "oracle", "emc_oracle.c"), "-lm"])
        except (OSError, subprocess.CalledProcessError) as e:
            pytest.skip(f"no sanitizer-capable gcc here: {e}")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
                   OMP_NUM_THREADS="1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert r.stdout.startswith("ok 25 ")
