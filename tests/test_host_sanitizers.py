"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The 1D element tables, the preconditioner eigenbasis, the wall projector and the space-time time
tables are built on the host in plain C++ (`csrc/pd_tables.cpp`). This test compiles that file with
g++ and `-fsanitize=address,undefined -fno-sanitize-recover=all` together with a small driver that
builds every supported degree (and the rejected ones) and checks the invariants each table must
satisfy, so an out-of-bounds access, an uninitialised read caught by UBSan or a wrong invariant
fails here without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_05806_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <string>
#include "pd_tables.h"

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { std::printf(__VA_ARGS__); std::printf("\n"); ++fails; } } while (0)

int main() {
  std::string err;
  for (int N = -1; N <= pdh::kMaxN + 1; ++N) {
    pdh::Table1D t;
    const bool ok = pdh::build_table(N, &t, &err);
    if (N < 0 || N > pdh::kMaxN) { CHECK(!ok, "degree %d accepted", N); continue; }
    CHECK(ok, "degree %d rejected: %s", N, err.c_str());
    const int n = t.n;
    double ws = 0.0, tr = 0.0, tro = 0.0;
    for (int i = 0; i < n; ++i) {
      ws += t.w[i];
      tr += t.Pnull[i * n + i];
      tro += t.PnullOdd[i * n + i];
    }
    CHECK(std::fabs(ws - 1.0) < 1e-14, "N=%d weights sum %.17g", N, ws);
    CHECK(std::fabs(tr - t.nnull) < 1e-10, "N=%d trace(Pnull) %.17g vs %d", N, tr, t.nnull);
    CHECK(std::fabs(tro - t.nnull_odd) < 1e-10, "N=%d trace(PnullOdd) %.17g vs %d", N, tro, t.nnull_odd);
    CHECK(t.nnull == (N % 2 == 0 ? 1 : 2), "N=%d nnull %d", N, t.nnull);
    CHECK(t.nnull_odd == (N % 2 == 0 ? 0 : 1), "N=%d nnull_odd %d", N, t.nnull_odd);
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        // L = R^T, C symmetric, V^T M V = I, C V = M V diag(lam); mirror symmetry of the
        // blocks under the node reversal J (R = J L J, C = J C J), which the even/odd form of
        // the device line operator relies on
        CHECK(t.Lb[p * n + q] == t.Rb[q * n + p], "N=%d L != R^T", N);
        CHECK(std::fabs(t.Rb[p * n + q] - t.Lb[(n - 1 - p) * n + (n - 1 - q)]) <= 1e-13 * (1.0 + std::fabs(t.Lb[p * n + q])),
              "N=%d R != J L J at (%d,%d)", N, p, q);
        CHECK(std::fabs(t.Cb[p * n + q] - t.Cb[(n - 1 - p) * n + (n - 1 - q)]) <= 1e-12 * (1.0 + std::fabs(t.Cb[p * n + q])),
              "N=%d C != J C J at (%d,%d)", N, p, q);
        CHECK(std::fabs(t.Cb[p * n + q] - t.Cb[q * n + p]) <= 1e-12 * std::fabs(t.Cb[p * n + p]) + 1e-12,
              "N=%d C not symmetric", N);
        double g = 0.0, cv = 0.0;
        for (int m = 0; m < n; ++m) {
          g += t.PV[m * n + p] * t.w[m] * t.PV[m * n + q];
          cv += t.Cb[p * n + m] * t.PV[m * n + q];
        }
        CHECK(std::fabs(g - (p == q ? 1.0 : 0.0)) < 1e-10, "N=%d V^T M V (%d,%d) = %.3e", N, p, q, g);
        const double mv = t.w[p] * t.PV[p * n + q] * t.Plam[q];
        CHECK(std::fabs(cv - mv) <= 1e-9 * (1.0 + std::fabs(mv)), "N=%d C V != M V lam", N);
      }
  }
  for (int M = -1; M <= pdh::kMaxM + 1; ++M) {
    pdh::TimeTable tt;
    const bool ok = pdh::build_time_table(M, &tt, &err);
    if (M < 0 || M > pdh::kMaxM) { CHECK(!ok, "time degree %d accepted", M); continue; }
    CHECK(ok, "time degree %d rejected: %s", M, err.c_str());
    const int m = tt.m;
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += tt.Ainv[p * m + k] * tt.At[k * m + q];
        CHECK(std::fabs(s - (p == q ? 1.0 : 0.0)) < 1e-11, "M=%d Ainv At (%d,%d) = %.3e", M, p, q, s);
      }
  }
  std::printf("host table checks: %d failures\n", fails);
  return fails == 0 ? 0 : 1;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_tables_under_asan_ubsan(tmp_path):
    drv = tmp_path / "drv.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, str(drv), os.path.join(CSRC, "pd_tables.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the process may have other preloaded libraries ahead of ASan
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
