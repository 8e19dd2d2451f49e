"""Host sanitizer run of the oracle's C integrals: oracle/mdints.c built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, runtimes linked
statically, every report fatal) under a small C driver that calls each of
its entry points once on water in 6-31G* (s, p and Cartesian d shells).  The
run must end cleanly, and its results must equal those of the library as
the oracle loads it, so the sanitized build checks the code the tests use."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import inputs
import oracle
from oracle import rhf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "native", "oracle_san_main.c")
SRC = os.path.join(ROOT, "oracle", "mdints.c")


@pytest.fixture(scope="module")
def san_exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path_factory.mktemp("san") / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-static-libasan", "-static-libubsan", "-o", exe, DRIVER, SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    return exe


def _write_input(path, b, P, W):
    ints = [np.array([b["nsh"], b["nbf"], len(b["Z"]), len(b["exps"])], np.int32)]
    ints += [np.ascontiguousarray(b[k], np.int32) for k in ("l", "atom", "nprim", "pofs", "bf", "Z")]
    dbl = [np.ascontiguousarray(b[k], np.float64).ravel() for k in ("exps", "coefs", "xyz")]
    dbl += [np.ascontiguousarray(P).ravel(), np.ascontiguousarray(W).ravel()]
    with open(path, "wb") as f:
        for a in ints + dbl:
            f.write(a.tobytes())


def _reference(b, P, W):
    """The same calls, in the driver's order, on the oracle's own build."""
    lib = rhf._c()
    p = rhf._p
    args = rhf._bargs(b)
    n, nsh, nat = b["nbf"], b["nsh"], len(b["Z"])
    xyz = p(b["xyz"])
    Zi = np.ascontiguousarray(b["Z"], np.int32)
    out = []
    for k in range(64):
        out.append(rhf.boys(16, 0.37 * k * k / 8.0))
    out += list(rhf.one_electron(b))
    out.append(rhf.eri_tensor(b))
    a, c1 = nsh - 1, 1 if nsh > 1 else 0
    blk, der = rhf.eri_quartet(b, a, a, 0, c1, deriv=True)
    out += [blk, der]
    Q = rhf.schwarz(b)
    out.append(Q)
    J, K, cnt = rhf.jk(b, P, 1e-12, Q)
    out += [np.array([cnt], float), J, K]
    Js, Ks = np.zeros((n, n)), np.zeros((n, n))
    cnt = lib.or_jk_sample(*args, xyz, p(Q), ctypes.c_double(1e-12), p(P), ctypes.c_int(3),
                           ctypes.c_int(2), p(Js), p(Ks))
    out += [np.array([cnt], float), Js, Ks]
    pairs = [(i, j) for i in range(nsh) for j in range(i + 1)]
    pa = np.array([i for i, _ in pairs], np.int32)
    pb = np.array([j for _, j in pairs], np.int32)
    Jp, Kp = np.zeros((n, n)), np.zeros((n, n))
    lib.or_jk_pairs(*args, xyz, p(Q), ctypes.c_double(1e-12), p(P), ctypes.c_int(len(pairs)),
                    p(pa), p(pb), p(Jp), p(Kp))
    out += [Jp, Kp]
    g = np.zeros((nat, 3))
    lib.or_grad_2e_kx(*args, xyz, ctypes.c_int(nat), p(Q), ctypes.c_double(1e-12), p(P),
                      ctypes.c_double(0.2), p(g))
    out.append(g)
    amask = np.zeros(nat, np.int32)
    amask[::2] = 1
    ga = np.zeros((nat, 3))
    lib.or_grad_2e_atoms(*args, xyz, ctypes.c_int(nat), p(Q), ctypes.c_double(1e-12), p(P),
                         p(amask), p(ga))
    out.append(ga)
    g1, g1a = np.zeros((nat, 3)), np.zeros((nat, 3))
    lib.or_grad_1e(*args, ctypes.c_int(nat), xyz, p(Zi), p(P), p(W), p(g1))
    lib.or_grad_1e_atoms(*args, ctypes.c_int(nat), xyz, p(Zi), p(P), p(W), p(amask), p(g1a))
    out += [g1, g1a]
    return [np.asarray(x, float).ravel() for x in out]


def test_oracle_integrals_clean_under_asan_and_ubsan(san_exe, tmp_path):
    z, x = inputs.water_cluster(1, 4)
    b = oracle.build_basis(inputs.load_basis("6-31g*"), z, x)
    n = b["nbf"]
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, n))
    P = np.ascontiguousarray(0.1 * (A + A.T))
    A = rng.standard_normal((n, n))
    W = np.ascontiguousarray(0.05 * (A + A.T))
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(fin, b, P, W)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([san_exe, fin, fout], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    got = np.fromfile(fout, np.float64)
    ref = _reference(b, P, W)
    assert got.size == sum(a.size for a in ref)
    o = 0
    for k, a in enumerate(ref):
        seg = got[o:o + a.size]
        o += a.size
        assert np.allclose(seg, a, rtol=1e-12, atol=1e-13), k


def test_the_sanitizer_flags_catch_an_overrun(tmp_path):
    """The same flags on a planted one-past-the-end read: the run must stop
    with a sanitizer report (the object-size check or AddressSanitizer,
    whichever sees it first), so a clean run above means something."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    src, exe = tmp_path / "bad.c", str(tmp_path / "bad")
    src.write_text("#include <stdlib.h>\n"
                   "int main(int c, char** v) { int* a = malloc(4 * sizeof(int));\n"
                   "  for (int i = 0; i < 4; ++i) a[i] = i;\n"
                   "  int s = a[3 + c]; free(a); return s == 12345; }\n")
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-static-libasan", "-static-libubsan", "-o", exe, str(src)],
                   check=True, capture_output=True, text=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr or "runtime error" in r.stderr
