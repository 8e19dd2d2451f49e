"""CPU check of the generated Obara-Saika/HRR code (no GPU).

The generator emits straight-line device functions; here their bodies are
translated line by line into Python (fma(a,b,c) -> a*b+c) and evaluated on
uncontracted primitive quartets, then compared with the oracle's
McMurchie-Davidson integrals and centre derivatives.  This pins the
generated recurrences of every class, including the heavy d classes, without
a device.
"""

import math
import os
import re
import sys

import numpy as np
import pytest

import oracle

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1601_02713_amd", "csrc")
sys.path.insert(0, CSRC)
import gen_eri  # noqa: E402


def _body(code, fname):
    """Statements of function `fname` in generated code, as Python lines."""
    start = code.index(f" {fname}(")
    brace = code.index("{", start)
    depth, i = 0, brace
    while True:
        if code[i] == "{":
            depth += 1
        elif code[i] == "}":
            depth -= 1
            if depth == 0:
                break
        i += 1
    out = []
    for ln in code[brace + 1:i].split(";"):
        ln = ln.strip()
        if not ln or ln.startswith("//"):
            continue
        ln = re.sub(r"^const R ", "", ln)
        if re.match(r"^R \w+\[\d+\]$", ln):
            nm, sz = re.match(r"^R (\w+)\[(\d+)\]$", ln).groups()
            out.append(f"{nm} = [0.0]*{sz}")
            continue
        ln = re.sub(r"\bR\(", "(", ln)
        ln = re.sub(r"\bdouble\(", "(", ln)
        out.append(ln)
    return out


def _fma(a, b, c):
    return a * b + c


def _boys(L, T):
    return oracle.boys(L, T)


def _prim_inputs(sh):
    """Primitive-quartet inputs in the kernel's conventions for shells
    sh = [(l, alpha, centre)] * 4 (unit contraction coefficients)."""
    (la, a, A), (lb, b, B), (lc, c, C), (ld, d, D) = sh
    p, q = a + b, c + d
    P = (a * A + b * B) / p
    Q = (c * C + d * D) / q
    Kab = math.exp(-a * b / p * np.dot(A - B, A - B))
    Kcd = math.exp(-c * d / q * np.dot(C - D, C - D))
    Cab = 5.9149671727956128778 * Kab / p
    Ccd = 5.9149671727956128778 * Kcd / q
    rho = p * q / (p + q)
    PQ = P - Q
    T = rho * np.dot(PQ, PQ)
    L = la + lb + lc + ld
    env = dict(PAx=(P - A)[0], PAy=(P - A)[1], PAz=(P - A)[2],
               QCx=(Q - C)[0], QCy=(Q - C)[1], QCz=(Q - C)[2],
               WPx=-q / (p + q) * PQ[0], WPy=-q / (p + q) * PQ[1], WPz=-q / (p + q) * PQ[2],
               WQx=p / (p + q) * PQ[0], WQy=p / (p + q) * PQ[1], WQz=p / (p + q) * PQ[2],
               oo2p=0.5 / p, oo2q=0.5 / q, oo2pq=0.5 / (p + q), rho_p2=0.5 / p * q / (p + q),
               rho_q2=0.5 / q * p / (p + q), ABx=(A - B)[0], ABy=(A - B)[1], ABz=(A - B)[2],
               CDx=(C - D)[0], CDy=(C - D)[1], CDz=(C - D)[2], wa=2 * a, wb=2 * b, wc=2 * c,
               fma=_fma, w=1.0)
    pref = Cab * Ccd / math.sqrt(p + q)
    return env, pref, T, L


def _oracle_quartet(sh, deriv=False):
    """Oracle block for single normalised primitives (coefficient = radial norm)."""
    l, atom, nprim, pofs, bf, exps, coefs = [], [], [], [], [], [], []
    nbf = 0
    for k, (ll, al, X) in enumerate(sh):
        l.append(ll); atom.append(k); nprim.append(1); pofs.append(k); bf.append(nbf)
        exps.append(al)
        coefs.append(1.0)
        nbf += (ll + 1) * (ll + 2) // 2
    i32 = lambda v: np.array(v, np.int32)
    b = dict(l=i32(l), atom=i32(atom), nprim=i32(nprim), pofs=i32(pofs), bf=i32(bf),
             exps=np.array(exps), coefs=np.array(coefs), nbf=nbf, nsh=4,
             xyz=np.array([s[2] for s in sh]), Z=i32([1] * 4))
    return oracle.eri_quartet(b, 0, 1, 2, 3, deriv=deriv)


RNG = np.random.default_rng(3)


def _rand_shells(ls):
    return [(l, RNG.uniform(0.3, 2.5), RNG.uniform(-1.0, 1.0, 3)) for l in ls]


ENERGY_CLASSES = ["1110", "2100", "2111", "2211", "2222"]


@pytest.mark.parametrize("tag", ENERGY_CLASSES)
def test_generated_energy_class(tag):
    la, lb, lc, ld = map(int, tag)
    fn_v, nacc, _, code_v = gen_eri.gen_vrr(la, la + lb, lc, lc + ld)
    fn_h, _, _, code_h = gen_eri.gen_hrr(la, lb, lc, ld)
    sh = _rand_shells([la, lb, lc, ld])
    env, pref, T, L = _prim_inputs(sh)
    env["F"] = list(_boys(L, T) * pref)
    env["acc"] = [0.0] * nacc
    exec("\n".join(_body(code_v, fn_v)), env)
    env["out"] = [0.0] * (gen_eri.ncart(la) * gen_eri.ncart(lb) * gen_eri.ncart(lc) * gen_eri.ncart(ld))
    exec("\n".join(_body(code_h, fn_h)), env)
    got = np.array(env["out"])
    ref = _oracle_quartet(sh).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


GRAD_CLASSES = ["1000", "1100", "1111", "2010", "2110", "2121", "2211", "2221", "2222"]


@pytest.mark.parametrize("tag", GRAD_CLASSES)
def test_generated_gradient_class(tag):
    la, lb, lc, ld = map(int, tag)
    sets, sizes, _, _, code = gen_eri.gen_grad(la, lb, lc, ld)
    sh = _rand_shells([la, lb, lc, ld])
    env, pref, T, L = _prim_inputs(sh)
    env["F"] = list(_boys(L + 1, T) * pref)
    nout = gen_eri.ncart(la) * gen_eri.ncart(lb) * gen_eri.ncart(lc) * gen_eri.ncart(ld)
    G = RNG.standard_normal(nout)
    env["G"] = list(G)
    env["g"] = [0.0] * 9
    env["one"] = 1.0
    if la + lb + lc + ld >= 6:
        for X in "ABC":
            exec("\n".join(_body(code, f"gprim{X}_{tag}")), env)
    else:
        for s in sets:
            env[s[0]] = [0.0] * sizes[s[0]]
        exec("\n".join(_body(code, f"gvrr_{tag}")), env)
        exec("\n".join(_body(code, f"gcon_{tag}")), env)
    got = np.array(env["g"])
    _, der = _oracle_quartet(sh, deriv=True)
    # oracle blocks are for normalised functions; the generated contraction
    # applies the component norms itself, with unit radial coefficients here
    ref = np.array([np.sum(G * der[cen, dd].ravel()) for cen in range(3) for dd in range(3)])
    assert np.abs(got - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()), (got, ref)


# ------------------------------------------------ cooperative node programs
import gen_coop  # noqa: E402


def _contracted_oracle(shells, deriv=False):
    """Oracle block for shells [(l, [alphas], [coefs], centre)] with the given
    raw contraction coefficients (no renormalisation)."""
    l, atom, nprim, pofs, bf, exps, coefs = [], [], [], [], [], [], []
    nbf = 0
    for k, (ll, al, co, X) in enumerate(shells):
        l.append(ll); atom.append(k); nprim.append(len(al)); pofs.append(len(exps)); bf.append(nbf)
        exps += list(al)
        coefs += list(co)
        nbf += (ll + 1) * (ll + 2) // 2
    i32 = lambda v: np.array(v, np.int32)
    b = dict(l=i32(l), atom=i32(atom), nprim=i32(nprim), pofs=i32(pofs), bf=i32(bf),
             exps=np.array(exps), coefs=np.array(coefs), nbf=nbf, nsh=4,
             xyz=np.array([s[3] for s in shells]), Z=i32([1] * 4))
    return oracle.eri_quartet(b, 0, 1, 2, 3, deriv=deriv)


def _program_inputs(shells, Lmax):
    """Per-primitive-quartet Boys values and the 27 scalars of gen_coop."""
    Fs, scs = [], []
    (la, aa, ca, A), (lb, ab, cb, B), (lc, ac, cc, C), (ld, ad, cd, D) = shells
    for ia, a in enumerate(aa):
        for ib, b in enumerate(ab):
            for ic, c in enumerate(ac):
                for id_, d in enumerate(ad):
                    sh = [(la, a, A), (lb, b, B), (lc, c, C), (ld, d, D)]
                    env, pref, T, _ = _prim_inputs(sh)
                    pref *= ca[ia] * cb[ib] * cc[ic] * cd[id_]
                    Fs.append(list(_boys(Lmax, T) * pref))
                    sc = [0.0] * gen_coop.NSEL
                    for nm, k in gen_coop.SEL.items():
                        sc[k] = 1.0 if nm == "one" else env[nm]
                    scs.append(sc)
    return Fs, scs


def _rand_contracted(ls, nprim):
    out = []
    for l, k in zip(ls, nprim):
        out.append((l, list(RNG.uniform(0.3, 2.5, k)), list(RNG.uniform(0.2, 1.0, k)),
                    RNG.uniform(-1.0, 1.0, 3)))
    return out


@pytest.mark.parametrize("tag,nprim", [("0000", (3, 2, 1, 2)), ("1010", (2, 1, 2, 1)),
                                       ("2121", (2, 1, 1, 2)), ("2211", (1, 2, 2, 1)),
                                       ("2220", (1, 1, 1, 2)), ("2222", (1, 1, 1, 1))])
def test_cooperative_energy_program(tag, nprim):
    la, lb, lc, ld = map(int, tag)
    # the tables as the kernels decode them (packed node/term words)
    prog = gen_coop.packed(gen_coop.energy_program(la, lb, lc, ld))
    sh = _rand_contracted([la, lb, lc, ld], nprim)
    Fs, scs = _program_inputs(sh, la + lb + lc + ld)
    got = np.array(gen_coop.interpret(prog, Fs, scs, scs[0]))
    ref = _contracted_oracle(sh).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("tag,nprim", [("0000", (2, 2, 1, 2)), ("1000", (2, 1, 2, 1)),
                                       ("2010", (1, 2, 2, 1)), ("1111", (2, 2, 2, 2)),
                                       ("2111", (1, 2, 2, 1)), ("2121", (2, 1, 1, 2)),
                                       ("2222", (1, 1, 1, 1))])
def test_cooperative_gradient_program(tag, nprim):
    la, lb, lc, ld = map(int, tag)
    prog = gen_coop.packed(gen_coop.grad_program(la, lb, lc, ld))
    sh = _rand_contracted([la, lb, lc, ld], nprim)
    Fs, scs = _program_inputs(sh, la + lb + lc + ld + 1)
    nout = gen_eri.ncart(la) * gen_eri.ncart(lb) * gen_eri.ncart(lc) * gen_eri.ncart(ld)
    G = RNG.standard_normal(nout)
    got = np.array(gen_coop.interpret(prog, Fs, scs, scs[0], grad_G=list(G)))
    _, der = _contracted_oracle(sh, deriv=True)
    ref = np.array([np.sum(G * der[cen, dd].ravel()) for cen in range(3) for dd in range(3)])
    assert np.abs(got - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()), (got, ref)


@pytest.mark.parametrize("tag", ["0000", "2110", "2222"])
def test_cooperative_tables_pack_losslessly(tag):
    """Packed node/term/contraction words decode to the generated tables."""
    la, lb, lc, ld = map(int, tag)
    for prog in (gen_coop.energy_program(la, lb, lc, ld), gen_coop.grad_program(la, lb, lc, ld)):
        q = gen_coop.packed(prog)
        for ph in ("vrr", "hrr"):
            assert [list(x) for x in q[ph]] == [list(x) for x in prog[ph]]
        for k in ("con_slot", "con_G", "con_g", "con_c"):
            if k in prog:
                assert list(q[k]) == list(prog[k])
        nt = gen_coop.threads_per_block(prog, "con_c" in prog)
        assert nt % 64 == 0 and 64 <= nt <= 512
