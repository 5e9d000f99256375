"""The kernels compile for gfx950 without register spills to scratch memory: a spill
turns a bandwidth-bound kernel's registers into extra memory traffic."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_04421_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
@pytest.mark.parametrize("src", sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")))
def test_no_scratch_spills(src, tmp_path):
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-c", "-O3", "-std=c++17", "-fPIC",
           "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, src), "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    name, spills = None, []
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            spills.append((name, int(m.group(1))))
    assert not spills, spills


_ORDER_PROBE = r"""
#include "abm_internal.h"
#include <cstdio>
#include <vector>
using namespace abm;
int main() {
  // xcd_block: a permutation of [0, G) that gives each XCD's workgroups (b mod 8)
  // consecutive indices, in the order the dispatcher starts them
  for (int G = 1; G <= 3000; ++G) {
    std::vector<int> seen(G, 0);
    for (int b = 0; b < G; ++b) {
      const int g = xcd_block(b, G);
      if (g < 0 || g >= G || seen[g]++) { std::printf("xcd_block G=%d b=%d\n", G, b); return 1; }
      if (b >= 8 && xcd_block(b, G) != xcd_block(b - 8, G) + 1) { std::printf("order G=%d b=%d\n", G, b); return 1; }
    }
  }
  // xcd_interleave: every batch exactly once, each workgroup at most bpw of them, and
  // the workgroups of one XCD started together on neighbouring batches
  const int nbts[] = {1, 2, 7, 8, 9, 63, 100, 1023, 4096, 48829};
  for (int nbt : nbts)
    for (int bpw = 1; bpw <= 16; ++bpw) {
      const int G = (nbt + bpw - 1) / bpw;
      std::vector<int> seen(nbt, 0);
      for (int b = 0; b < G; ++b) {
        const Interleave il = xcd_interleave(b, G, bpw, nbt);
        if (il.count > bpw) { std::printf("count nbt=%d bpw=%d b=%d\n", nbt, bpw, b); return 1; }
        for (int j = 0; j < il.count; ++j) {
          const int bt = il.first + j * il.stride;
          if (bt < 0 || bt >= nbt || seen[bt]++) { std::printf("cover nbt=%d bpw=%d b=%d\n", nbt, bpw, b); return 1; }
        }
        if (b >= 8 && il.count > 0 && il.first != xcd_interleave(b - 8, G, bpw, nbt).first + 1) {
          std::printf("neighbours nbt=%d bpw=%d b=%d\n", nbt, bpw, b); return 1;
        }
      }
      for (int bt = 0; bt < nbt; ++bt)
        if (seen[bt] != 1) { std::printf("missed nbt=%d bpw=%d bt=%d\n", nbt, bpw, bt); return 1; }
    }
  std::printf("ok\n");
  return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_xcd_workgroup_orders_cover_every_index_once(tmp_path):
    """The workgroup orders of the generation pass and the partition scatters: the
    XCD-aware numbering is a permutation, and the interleaved batch ranges of the
    level-1 scatter take every batch exactly once (host build of the same functions)."""
    src = tmp_path / "order.hip"
    src.write_text(_ORDER_PROBE)
    exe = tmp_path / "order"
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O1", "-std=c++17", "--cuda-host-only",
           "-x", "hip", "-I", os.path.join(ROOT, "include"), "-I", CSRC, str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
