"""The host side of the C ABI (argument validation, the analysis of run-time
bases, workspace planning) built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven through its entry points without a GPU.

csrc/api.hip is compiled with the sanitizers on its host code only (device
code cannot be instrumented) and linked with the library's other objects and
a small C++ driver.  Every call the driver makes either fails validation
before any HIP call or, for a run-time basis that passes the analysis, fails
at the device allocation (no GPU here); the driver checks each return code.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "lbmrv")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <vector>
#include "lbmrv.h"

static int fails = 0;
#define EXPECT(cond) do { if (!(cond)) { std::printf("FAILED line %d: %s\n", __LINE__, #cond); ++fails; } } while (0)

int main() {
  const double s9[9] = {0, 0, 0, 1.4, 1.7, 1.7, 1.2, 1.2, 1.4};
  const int64_t d2[2] = {33, 17}, d3[3] = {9, 8, 7};
  std::vector<double> s19(19, 1.3), s27(27, 1.3);
  for (int k = 0; k <= 3; ++k) s19[k] = s27[k] = 0.0;
  lbmrv_ctx* c = nullptr;
  // creation and its validation
  EXPECT(lbmrv_create(&c, LBMRV_D2Q9, LBMRV_BASIS_DEFAULT, 1.0, s9, d2, LBMRV_F32DEV, 1.0) == LBMRV_OK);
  int64_t q = 0, d = 0, n = 0, b = 0;
  EXPECT(lbmrv_info(c, &q, &d, &n, &b) == LBMRV_OK && q == 9 && d == 2 && n == 33 * 17 && b == 4);
  EXPECT(lbmrv_set_streaming(c, LBMRV_STREAM_AA) == LBMRV_OK);
  EXPECT(lbmrv_set_streaming(c, 7) == LBMRV_ERR_INVALID_ARG);
  const double wu[18] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0.05, 0, 0, 0, 0, 0, 0, 0, 0};
  EXPECT(lbmrv_set_walls(c, 0xC, wu, 1.0) == LBMRV_OK);
  EXPECT(lbmrv_set_walls(c, 1u << 4, nullptr, 1.0) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_set_equilibrium(c, LBMRV_EQ_MAXWELLIAN) == LBMRV_OK);
  EXPECT(lbmrv_set_block_order(c, LBMRV_ORDER_XCD) == LBMRV_OK);
  double bad[9] = {0, 0.1, 0, 1, 1, 1, 1, 1, 1};
  EXPECT(lbmrv_set_rates(c, bad) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_set_rates(c, s9) == LBMRV_OK);
  EXPECT(lbmrv_step(c, nullptr, nullptr, LBMRV_UT_FLUID, 1.0, nullptr, 1, nullptr) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_step(c, (void*)4096, (void*)8192, 9, 1.0, nullptr, 1, nullptr) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_step(c, (void*)4098, (void*)8192, LBMRV_UT_ZERO, 1.0, nullptr, 1, nullptr) == LBMRV_ERR_ALIGNMENT);
  EXPECT(lbmrv_conservation(c, (void*)4096, nullptr, nullptr) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_adjoint_workspace_bytes(c, 2000, 100) > 0);
  EXPECT(lbmrv_adjoint_workspace_bytes(c, 0, 100) == 0);
  EXPECT(lbmrv_conservation_noalloc(c, (void*)4096, (double*)4097, nullptr) == LBMRV_ERR_ALIGNMENT);
  lbmrv_destroy(c);
  // grids and arguments that creation rejects
  const int64_t zero[2] = {0, 8}, big[3] = {4096, 4096, 256};
  EXPECT(lbmrv_create(&c, LBMRV_D2Q9, LBMRV_BASIS_DEFAULT, 1.0, s9, zero, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG && !c);
  EXPECT(lbmrv_create(&c, LBMRV_D3Q19, LBMRV_BASIS_DEFAULT, 1.0, s19.data(), big, LBMRV_F16DEV, 1.0) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_create(&c, LBMRV_D3Q19, LBMRV_BASIS_GEIER, 1.0, s19.data(), d3, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_create(&c, LBMRV_D3Q27, LBMRV_BASIS_DEFAULT, NAN, s27.data(), d3, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
  EXPECT(lbmrv_create(&c, LBMRV_D3Q27, LBMRV_BASIS_DEFAULT, 1.0, s27.data(), d3, LBMRV_F64, 1.0) == LBMRV_OK);
  EXPECT(lbmrv_adjoint_workspace_bytes(c, 23, 7) > 0);
  lbmrv_destroy(c);
  // run-time bases: analysed on the host, then the table upload needs a GPU
  // D2Q9 raw powers of |xi|^2 (the span of eq. (mom))
  {
    const int32_t pot[] = {0, 1, 2, 3, 3, 4, 4, 5, 6, 6, 7, 7, 8, 8, 8};
    const int32_t ex[] = {0,0,0, 1,0,0, 0,1,0, 2,0,0, 0,2,0, 2,0,0, 0,2,0, 1,1,0, 3,0,0, 1,2,0,
                          2,1,0, 0,3,0, 4,0,0, 2,2,0, 0,4,0};
    const double co[] = {1, 1, 1, 1, 1, 1, -1, 1, 1, 1, 1, 1, 1, 2, 1};
    lbmrv_poly_basis pb{15, pot, ex, co};
    const int rc = lbmrv_create_custom(&c, LBMRV_D2Q9, &pb, 1.0, s9, d2, LBMRV_F32, 1.0);
    EXPECT(rc == LBMRV_OK || rc == LBMRV_ERR_HIP);
    if (rc == LBMRV_OK) lbmrv_destroy(c);
    // the same with the conserved polynomial 1 scaled: rejected by the analysis
    const double co2[] = {2, 1, 1, 1, 1, 1, -1, 1, 1, 1, 1, 1, 1, 2, 1};
    lbmrv_poly_basis pb2{15, pot, ex, co2};
    EXPECT(lbmrv_create_custom(&c, LBMRV_D2Q9, &pb2, 1.0, s9, d2, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
    // a polynomial outside every built-in span (xi_x^4 alone in place of the last one)
    const int32_t pot3[] = {0, 1, 2, 3, 3, 4, 4, 5, 6, 6, 7, 7, 8};
    const double co3[] = {1, 1, 1, 1, 1, 1, -1, 1, 1, 1, 1, 1, 1};
    lbmrv_poly_basis pb3{13, pot3, ex, co3};
    EXPECT(lbmrv_create_custom(&c, LBMRV_D2Q9, &pb3, 1.0, s9, d2, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
    // exponents out of range and a missing polynomial
    const int32_t ex4[] = {9,0,0, 1,0,0, 0,1,0, 2,0,0, 0,2,0, 2,0,0, 0,2,0, 1,1,0, 3,0,0, 1,2,0,
                           2,1,0, 0,3,0, 4,0,0, 2,2,0, 0,4,0};
    lbmrv_poly_basis pb4{15, pot, ex4, co};
    EXPECT(lbmrv_create_custom(&c, LBMRV_D2Q9, &pb4, 1.0, s9, d2, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
    lbmrv_poly_basis pb5{5, pot, ex, co};
    EXPECT(lbmrv_create_custom(&c, LBMRV_D2Q9, &pb5, 1.0, s9, d2, LBMRV_F32, 1.0) == LBMRV_ERR_INVALID_ARG);
  }
  // D3Q27 monomials (the default span), given one by one
  {
    std::vector<int32_t> pot, ex;
    std::vector<double> co;
    const int e27[27][3] = {{0,0,0},{1,0,0},{0,1,0},{0,0,1},{2,0,0},{0,2,0},{0,0,2},{1,1,0},{0,1,1},{1,0,1},
                            {1,2,0},{1,0,2},{2,1,0},{0,1,2},{2,0,1},{0,2,1},{1,1,1},{2,2,0},{2,0,2},{0,2,2},
                            {2,1,1},{1,2,1},{1,1,2},{2,2,1},{2,1,2},{1,2,2},{2,2,2}};
    for (int k = 0; k < 27; ++k) {
      pot.push_back(k);
      for (int a = 0; a < 3; ++a) ex.push_back(e27[k][a]);
      co.push_back(1.0);
    }
    lbmrv_poly_basis pb{27, pot.data(), ex.data(), co.data()};
    const int rc = lbmrv_create_custom(&c, LBMRV_D3Q27, &pb, 1.0, s27.data(), d3, LBMRV_F16DEV, 1.0);
    EXPECT(rc == LBMRV_OK || rc == LBMRV_ERR_HIP);
    if (rc == LBMRV_OK) lbmrv_destroy(c);
  }
  for (int code : {0, -1, -2, -4, -5, -6, -99}) EXPECT(lbmrv_strerror(code) != nullptr);
  int32_t cd[81];
  double w[27];
  EXPECT(lbmrv_lattice_tables(LBMRV_D3Q27, cd, w) == LBMRV_OK);
  EXPECT(lbmrv_lattice_tables(5, cd, w) == LBMRV_ERR_INVALID_ARG);
  std::printf("%s (%d failed)\n", fails ? "FAIL" : "OK", fails);
  return fails ? 1 : 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    objs = [o for o in sorted(glob.glob(os.path.join(BUILD, "lat_*.o")))]
    if not objs or not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("library objects not built (paper_1312_3297_amd/build.py) or hipcc missing")
    d = tmp_path_factory.mktemp("sanitized_abi")
    api_o = d / "api.o"
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    common = ["-O1", "-g", "-std=c++20", "-fPIC", "-I" + os.path.join(ROOT, "include"),
              "-Wno-unused-command-line-argument"]
    # sanitizers on the host code only: each -fsanitize= goes after -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [HIPCC, "--offload-arch=gfx950", "-fconstexpr-steps=100000000", "-fexperimental-new-constant-interpreter",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + common + san + \
          ["-c", os.path.join(ROOT, "paper_1312_3297_amd", "csrc", "api.hip"), "-o", str(api_o)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "unsupported" in r.stderr:
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr[-3000:]
    # the driver is plain C++, and the link is a host link with the HIP
    # runtime: both with the same clang that instrumented api.o
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    host_san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    drv_o = d / "driver.o"
    r = subprocess.run([clangxx] + common + host_san + ["-c", str(src), "-o", str(drv_o)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = d / "abi_driver"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
    link = [clangxx] + host_san + [str(drv_o), str(api_o)] + objs + \
        ["-L" + rocm_lib, "-lamdhip64", "-Wl,-rpath," + rocm_lib, "-o", str(exe)]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_host_abi_code_under_sanitizers(driver):
    # leaks of the HIP runtime at exit are not ours to chase; everything else aborts
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(driver)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "OK (0 failed)" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
