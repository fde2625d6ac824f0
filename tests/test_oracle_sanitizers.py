"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and driven through every entry point: models, sort,
potential, a whole step with both generators and the energy-correction
moves, the correction, diagnostics, the sampled orbit and the King profile.
Sizes 0, 1, 2 and 3001 cover the empty and ragged cases.  Any sanitizer
report aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include "cmc_oracle.h"
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int run(int64_t n, int lfsr_on) {
  size_t nn = (size_t)(n > 0 ? n : 1);
  double *r = malloc(nn * 8), *vr = malloc(nn * 8), *vt = malloc(nn * 8), *m = malloc(nn * 8);
  uint32_t *id = malloc(nn * 4);
  ora_plummer(n, 7, 1, r, vr, vt, m, id);
  int64_t *perm = malloc(nn * 8);
  ora_sort_perm(n, r, perm);
  double *sr = malloc(nn * 8), *svr = malloc(nn * 8), *svt = malloc(nn * 8), *sm = malloc(nn * 8);
  uint32_t *sid = malloc(nn * 4), *lfsr = malloc(4 * nn * 4);
  const uint32_t z0[4] = {12345u, 12345u, 12345u, 12345u};
  for (int64_t q = 0; q < n; ++q) {
    sr[q] = r[perm[q]]; svr[q] = vr[perm[q]]; svt[q] = vt[perm[q]]; sm[q] = m[perm[q]];
    sid[q] = id[perm[q]];
    ora_lfsr113_stream(z0, sid[q], lfsr + 4 * q);
  }
  double *phi = malloc(nn * 8), *mcum = malloc(nn * 8), *ssuf = malloc(nn * 8);
  double *moves = malloc(3 * nn * 8), *rn = malloc(nn * 8);
  ora_params p = {7, 0, 0.11, 0.03, 0.0, 10000, 1.2};
  ora_step_out o;
  ora_step_ex(n, sr, svr, svt, sm, sid, phi, mcum, &p, &o, moves, lfsr_on ? lfsr : NULL);
  int64_t k = o.n_after;
  ora_potential(k, sr, sm, phi, mcum, ssuf);
  ora_energy_correction(k, sr, sm, svr, svt, phi, moves);
  double out[11];
  ora_diagnostics(k, sr, svr, svt, sm, phi, mcum, out);
  if (k > 0) {
    int64_t idx[2] = {0, k - 1};
    ora_orbit_subset(k, sr, phi, mcum, ssuf, sm, svr, svt, sid, 7, 1, 10000, 1.2, 2, idx, rn);
    (void)ora_phi_at(k, sr, phi, mcum, ssuf, 0.5 * sr[k - 1]);
  }
  printf("n=%lld kept=%lld E=%g\n", (long long)n, (long long)k, out[2]);
  free(r); free(vr); free(vt); free(m); free(id); free(perm); free(sr); free(svr); free(svt);
  free(sm); free(sid); free(lfsr); free(phi); free(mcum); free(ssuf); free(moves); free(rn);
  return 0;
}

int main(void) {
  const int64_t sizes[4] = {0, 1, 2, 3001};
  for (int s = 0; s < 4; ++s)
    for (int g = 0; g < 2; ++g) run(sizes[s], g);
  double rk[4096], Wk[4096], Mk[4096], tail[3];
  int nodes = ora_king_profile(6.0, rk, Wk, Mk, 4096, tail);
  double r[500], vr[500], vt[500], m[500];
  uint32_t id[500];
  ora_king(500, 3, 6.0, 0, r, vr, vt, m, id);
  printf("king nodes=%d\nok\n", nodes);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    flags = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", *flags, "-I", os.path.join(ROOT, "oracle"), "-o", str(exe), str(src),
                    os.path.join(ROOT, "oracle", "cmc_oracle.c"), "-lm"], check=True)
    # verify_asan_link_order=0: the environment's own preloaded libraries, if
    # any, stay as they are
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stderr[-3000:]
    assert p.stdout.strip().endswith("ok"), p.stdout
    assert "runtime error" not in p.stderr, p.stderr[-3000:]
