"""LDS slot ownership of the two-half p = 128 transform (host checks, no GPU).

The p = 128 sweep parks one half of a frame in LDS slots and drops the leading
barriers of its half transforms.  That is race-free because each thread's first LDS
writes in a half transform go only to slots that no other thread touches between:
  * Half128::own_pair(t, k): the 16 values thread t reads in the last stage-C pass
    (and parks into, and writes first in the inverse);
  * Half128::a_slot(t, k, l) and Half128MF::a_slot(w, lane, cb, jj): the stage-A
    slots written first in the forward half and read last in the inverse.
Both kernels and this test use those same header functions, so the premise that is
checked here is the one the kernels rely on: for every function the slots of
different threads are disjoint, inside the LDS buffer, and 128-bit aligned where they
are accessed as pairs.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_00162_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "fft_frame.hpp"
#include "fft_mfma.hpp"
using namespace odp;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; std::printf(__VA_ARGS__); } } while (0)
int main() {
  const int T = Half128::T, LDS = Half128::LDS;
  std::vector<int> owner(LDS, -1);
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < 8; ++k) {
      const int i = Half128::own_pair(t, k);
      CHECK(i >= 0 && i + 1 < LDS, "own_pair(%d,%d)=%d outside\n", t, k, i);
      CHECK(i % 2 == 0, "own_pair(%d,%d)=%d not 16-byte aligned\n", t, k, i);
      for (int e = i; e < i + 2 && e >= 0 && e < LDS; ++e) {
        CHECK(owner[e] < 0 || owner[e] == t, "slot %d of threads %d and %d\n", e, owner[e], t);
        owner[e] = t;
      }
    }
  owner.assign(LDS, -1);
  for (int t = 0; t < T; ++t)
    for (int l = 0; l < 2; ++l)
      for (int k = 0; k < 8; ++k) {
        const int i = Half128::a_slot(t, k, l);
        CHECK(i >= 0 && i < LDS, "a_slot(%d,%d,%d)=%d outside\n", t, k, l, i);
        if (i < 0 || i >= LDS) continue;
        CHECK(owner[i] < 0, "stage-A slot %d of threads %d and %d\n", i, owner[i], t);
        owner[i] = t;
      }
  owner.assign(LDS, -1);
  for (int t = 0; t < Half128MF::T; ++t)
    for (int cb = 0; cb < 8; ++cb)
      for (int jj = 0; jj < 2; ++jj) {
        const int i = Half128MF::a_slot(t >> 6, t & 63, cb, jj);
        CHECK(i >= 0 && i < LDS, "MF a_slot(%d,%d,%d)=%d outside\n", t, cb, jj, i);
        if (i < 0 || i >= LDS) continue;
        CHECK(owner[i] < 0, "MF stage-A slot %d of threads %d and %d\n", i, owner[i], t);
        owner[i] = t;
      }
  std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
"""


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    return None


def test_two_half_transform_lds_slots_are_thread_private():
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "slots.hip")
        exe = os.path.join(d, "slots")
        with open(src, "w") as fh:
            fh.write(PROGRAM)
        cmd = [cc, "-std=c++17", "-O1", "--offload-host-only", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
               src, "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stdout + res.stderr
        run = subprocess.run([exe], capture_output=True, text=True)
        assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr
