"""The C oracles (oracle/fast/oracle_fast.c and oracle_tri.c) built with the
address and undefined-behaviour sanitizers and run on small ragged grids of
every lattice and u~ mode: no sanitizer report, and the results are Oracle A's.

A small C driver (written here, built with gcc) links both oracles, reads the
lattice tables and states from files this test writes, runs a few steps of
each form and writes the results back.  Without OpenMP (the pragmas are then
ignored), so the sanitizers see plain sequential code.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import fast, lattices
from oracle import scheme as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int d, q;
  const int *c;
  const double *w;
  int nterms;
  const int *term_poly;
  const int *term_exp;
  const double *term_coef;
  double la;
} lat_t;

int ob_run(const lat_t *L, const double *s, int mode, double alpha, const double *field, const int64_t *dims,
           int64_t nsteps, double *f, double *scratch, int nthreads);
void ot_run(const lat_t *L, const double *M0inv, const double *s, int mode, double alpha, const double *field,
            const int64_t *dims, int64_t nsteps, double *f, double *scratch, int nthreads);

static void *readall(const char *path, size_t *n) {
  FILE *fp = fopen(path, "rb");
  if (!fp) { perror(path); exit(2); }
  fseek(fp, 0, SEEK_END);
  long sz = ftell(fp);
  fseek(fp, 0, SEEK_SET);
  void *p = malloc(sz > 0 ? sz : 1);
  if (fread(p, 1, sz, fp) != (size_t)sz) exit(3);
  fclose(fp);
  *n = (size_t)sz;
  return p;
}

int main(int argc, char **argv) {
  /* argv: dir; files: hdr.i64 (d q nterms mode nsteps nx ny nz), c.i32, w.f64,
     tp.i32, te.i32, tc.f64, minv.f64, s.f64, field.f64, f.f64 */
  char path[4096];
  size_t n;
#define LOAD(var, type, name) snprintf(path, sizeof path, "%s/" name, argv[1]); type *var = readall(path, &n)
  LOAD(hdr, int64_t, "hdr.i64");
  LOAD(c, int, "c.i32");
  LOAD(w, double, "w.f64");
  LOAD(tp, int, "tp.i32");
  LOAD(te, int, "te.i32");
  LOAD(tc, double, "tc.f64");
  LOAD(minv, double, "minv.f64");
  LOAD(s, double, "s.f64");
  LOAD(field, double, "field.f64");
  LOAD(f0, double, "f.f64");
  const size_t fbytes = n;
  lat_t L = {(int)hdr[0], (int)hdr[1], c, w, (int)hdr[2], tp, te, tc, 1.0};
  const int mode = (int)hdr[3];
  const int64_t nsteps = hdr[4];
  const int64_t dims[3] = {hdr[5], hdr[6], hdr[7]};
  double *a = malloc(fbytes), *b = malloc(fbytes), *scr = malloc(fbytes);
  for (size_t i = 0; i < fbytes / sizeof(double); ++i) a[i] = b[i] = f0[i];
  if (ob_run(&L, s, mode, 0.8, field, dims, nsteps, a, scr, 1)) return 4;
  ot_run(&L, minv, s, mode, 0.8, field, dims, nsteps, b, scr, 1);
  snprintf(path, sizeof path, "%s/out.f64", argv[1]);
  FILE *fp = fopen(path, "wb");
  fwrite(a, 1, fbytes, fp);
  fwrite(b, 1, fbytes, fp);
  fclose(fp);
  free(a); free(b); free(scr);
  free(hdr); free(c); free(w); free(tp); free(te); free(tc); free(minv); free(s); free(field); free(f0);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("sanitized_oracle")
    src = d / "driver.c"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wno-unknown-pragmas", "-o", str(exe), str(src),
           os.path.join(ROOT, "oracle", "fast", "oracle_fast.c"), os.path.join(ROOT, "oracle", "fast", "oracle_tri.c"),
           "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("name", ["d2q9_paper", "d2q9_geier", "d3q19", "d3q27"])
@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID, A.FIELD])
def test_sanitized_oracles(driver, tmp_path, name, mode):
    lat = lattices.make(name)
    shape = (5, 7) if lat.d == 2 else (3, 4, 5)       # not a multiple of the 32-node batch
    rng = np.random.default_rng(20)
    rho = 1 + 0.05 * rng.standard_normal(shape)
    u = 0.1 * rng.uniform(-1, 1, (lat.d,) + shape)
    f = A.equilibrium(lat, rho, u) * (1 + 0.1 * rng.uniform(-1, 1, (lat.q,) + shape))
    s = np.concatenate([np.zeros(lat.d + 1), rng.uniform(0.6, 1.9, lat.q - lat.d - 1)])
    fld = rng.uniform(-0.3, 0.3, (lat.d,) + shape)
    tp, te, tc = fast._terms(lat, 1.0)
    dims = list(reversed(shape)) + [1] * (3 - len(shape))
    nsteps = 3
    np.array([lat.d, lat.q, len(tp), mode, nsteps] + dims, dtype=np.int64).tofile(tmp_path / "hdr.i64")
    lat.c.astype(np.int32).tofile(tmp_path / "c.i32")
    lat.w.astype(np.float64).tofile(tmp_path / "w.f64")
    tp.astype(np.int32).tofile(tmp_path / "tp.i32")
    te.astype(np.int32).tofile(tmp_path / "te.i32")
    tc.astype(np.float64).tofile(tmp_path / "tc.f64")
    fast._m0_inverse(lat, 1.0).astype(np.float64).tofile(tmp_path / "minv.f64")
    s.astype(np.float64).tofile(tmp_path / "s.f64")
    fld.astype(np.float64).tofile(tmp_path / "field.f64")
    f.astype(np.float64).tofile(tmp_path / "f.f64")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(driver), str(tmp_path)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    out = np.fromfile(tmp_path / "out.f64", dtype=np.float64).reshape((2,) + f.shape)
    ref = A.run(lat, f, s, nsteps, mode=mode, alpha=0.8, field=fld)
    for got in out:
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
