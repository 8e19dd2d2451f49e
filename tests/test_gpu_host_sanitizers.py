"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
on the GPU: tests/native/engine_san_main.c drives libbeadscf (host side
instrumented, device code as usual) through the C ABI over a ring polymer of
four beads of (H2O)2 in 6-31G*: SCF in both precisions and every density and
guess route, forces, MD steps with guess training, a checkpoint written and
loaded, B3LYP energies and forces, a string-method step, and refused calls.
The run must end without a sanitizer report and with every call as expected.
The instrumented build is made on the host by
``python -m paper_1601_02713_amd.build --host-sanitize``; without it the test
is skipped."""

import os
import subprocess

import pytest

import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1601_02713_amd", "_san", "engine_san")


@pytest.mark.skipif(not os.path.exists(EXE), reason="host sanitizer build not made")
def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    z, x = inputs.water_cluster(2, 31)
    xb = inputs.beads(z, x, 4, 31)
    geo = tmp_path / "geo.txt"
    geo.write_text(f"4 {len(z)}\n" + " ".join(map(str, z)) + "\n" +
                   " ".join(f"{v:.17g}" for v in xb.ravel()) + "\n")
    basis = os.path.join(ROOT, "inputs", "basis", "6-31gs.json")
    # the GPU runtime maps memory in the shadow gap and keeps allocations
    # until exit, so the gap stays unprotected and leak checking is off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([EXE, basis, str(geo), str(tmp_path / "run.ckpt")], env=env,
                       capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-4000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "failures 0" in r.stdout
