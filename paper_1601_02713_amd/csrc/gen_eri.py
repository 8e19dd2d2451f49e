#!/usr/bin/env python3
"""Generate straight-line Obara-Saika VRR + Head-Gordon-Pople HRR device code.

For every shell-quartet class (la lb|lc ld) with la >= lb, lc >= ld the
generator emits

  * ``vrr_<emin>_<emax>_<fmin>_<fmax>``: for one primitive quartet, the
    integrals [e0|f0]^(0) with emin <= |e| <= emax, fmin <= |f| <= fmax,
    built by the Obara-Saika vertical recurrences (Obara and Saika,
    J. Chem. Phys. 84, 3963 (1986), eqs. 39-40 in the form of Head-Gordon and
    Pople, J. Chem. Phys. 89, 5777 (1988)):

      [e+1_i,0|f0]^(m) = PA_i [e0|f0]^(m) + WP_i [e0|f0]^(m+1)
                         + e_i/(2p) ([e-1_i,0|f0]^(m) - rho/p [e-1_i,0|f0]^(m+1))
                         + f_i/(2(p+q)) [e0|f-1_i,0]^(m+1)
      [e0|f+1_i,0]^(m) = QC_i [e0|f0]^(m) + WQ_i [e0|f0]^(m+1)
                         + f_i/(2q) ([e0|f-1_i,0]^(m) - rho/q [e0|f-1_i,0]^(m+1))
                         + e_i/(2(p+q)) [e-1_i,0|f0]^(m+1)

    with [00|00]^(m) = prefactor * F_m(T) supplied by the caller;
    results are added with a weight into an accumulator array;
  * ``hrr_<la>_<lb>_<lc>_<ld>``: the horizontal recurrences
      (a,b+1_i| = (a+1_i,b| + AB_i (a,b|      |c,d+1_i) = |c+1_i,d) + CD_i |c,d)
    on contracted [e0|f0] producing the Cartesian block (ab|cd), row-major
    over (a, b, c, d) components in lexicographic order, each component
    scaled by 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!) so that every Cartesian
    function has unit norm.

Output: one header per class plus a common header; code is templated on the
arithmetic type R (double or float).  The generator also writes a FLOP table
(multiply-adds counted as 2) used for roofline accounting.
"""

from __future__ import annotations

import itertools
import json
import os
import sys

LMAX = 2  # s, p, d


def cart(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def ncart(l):
    return (l + 1) * (l + 2) // 2


def comp_norm(t):
    """1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!): unit norm for every Cartesian component."""
    d = 1
    for l in t:
        for k in range(2 * l - 1, 1, -2):
            d *= k
    return 1.0 / d ** 0.5


def shells_range(lo, hi):
    out = []
    for l in range(lo, hi + 1):
        out += cart(l)
    return out


def sub(t, i, k=1):
    u = list(t)
    u[i] -= k
    return tuple(u)


def add(t, i, k=1):
    u = list(t)
    u[i] += k
    return tuple(u)


class VRR:
    """Dependency-resolved, straight-line VRR for one (emin,emax,fmin,fmax)."""

    def __init__(self, emin, emax, fmin, fmax):
        self.emin, self.emax, self.fmin, self.fmax = emin, emax, fmin, fmax
        self.L = emax + fmax
        self.names = {}
        self.lines = []
        self.flops = 0
        self.targets = [(e, f) for e in shells_range(emin, emax) for f in shells_range(fmin, fmax)]

    def name(self, e, f, m):
        key = (e, f, m)
        if key in self.names:
            return self.names[key]
        if min(e) < 0 or min(f) < 0:
            return None
        se, sf = sum(e), sum(f)
        if se == 0 and sf == 0:
            nm = f"F[{m}]"
            self.names[key] = nm
            return nm
        terms = []  # (coef_expr or None, operand)
        if sf > 0:
            i = next(k for k in range(3) if f[k] > 0)
            f1 = sub(f, i)
            a = self.name(e, f1, m)
            b = self.name(e, f1, m + 1)
            terms.append((f"QC{'xyz'[i]}", a))
            terms.append((f"WQ{'xyz'[i]}", b))
            if f1[i] > 0:
                f2 = sub(f1, i)
                c = self.name(e, f2, m)
                d = self.name(e, f2, m + 1)
                terms.append((f"({f1[i]}*oo2q)", c))
                terms.append((f"(-{f1[i]}*rho_q2)", d))
            if e[i] > 0:
                g = self.name(sub(e, i), f1, m + 1)
                terms.append((f"({e[i]}*oo2pq)", g))
        else:
            i = next(k for k in range(3) if e[k] > 0)
            e1 = sub(e, i)
            a = self.name(e1, f, m)
            b = self.name(e1, f, m + 1)
            terms.append((f"PA{'xyz'[i]}", a))
            terms.append((f"WP{'xyz'[i]}", b))
            if e1[i] > 0:
                e2 = sub(e1, i)
                c = self.name(e2, f, m)
                d = self.name(e2, f, m + 1)
                terms.append((f"({e1[i]}*oo2p)", c))
                terms.append((f"(-{e1[i]}*rho_p2)", d))
        terms = [t for t in terms if t[1] is not None]
        nm = f"v{len(self.lines)}"
        expr = None
        for coef, opnd in terms:
            term = f"{coef}*{opnd}"
            if expr is None:
                expr = term
                self.flops += 1
            else:
                expr = f"fma({coef}, {opnd}, {expr})"
                self.flops += 2
        self.lines.append(f"const R {nm} = {expr};")
        self.names[key] = nm
        return nm

    def build(self):
        tnames = [self.name(e, f, 0) for e, f in self.targets]
        return tnames


def gen_vrr(emin, emax, fmin, fmax):
    v = VRR(emin, emax, fmin, fmax)
    tn = v.build()
    nacc = len(tn)
    body = ["  " + ln for ln in v.lines]
    acc_lines = [f"  acc[{k}] = fma(w, {n}, acc[{k}]);" for k, n in enumerate(tn)]
    flops = v.flops + 2 * nacc
    fn = f"vrr_{emin}_{emax}_{fmin}_{fmax}"
    code = [
        f"// [e0|f0]^(0), {emin}<=|e|<={emax}, {fmin}<=|f|<={fmax}: {nacc} targets, {flops} flops",
        "template <typename R>",
        f"__device__ __forceinline__ void {fn}(const R* __restrict__ F, const R PAx, const R PAy, const R PAz,",
        "    const R WPx, const R WPy, const R WPz, const R QCx, const R QCy, const R QCz,",
        "    const R WQx, const R WQy, const R WQz, const R oo2p, const R oo2q, const R oo2pq,",
        f"    const R rho_p2, const R rho_q2, const R w, R* __restrict__ acc) {{",
    ] + body + acc_lines + ["}", ""]
    return fn, nacc, flops, "\n".join(code)


def gen_hrr(la, lb, lc, ld):
    """(ab|cd) from contracted [e0|f0], e in [la, la+lb], f in [lc, lc+ld]."""
    E = shells_range(la, la + lb)
    Fs = shells_range(lc, lc + ld)
    eidx = {e: k for k, e in enumerate(E)}
    fidx = {f: k for k, f in enumerate(Fs)}
    nf = len(Fs)
    lines = []
    flops = 0
    names = {}

    def src(e, f):
        return f"acc[{eidx[e] * nf + fidx[f]}]"

    # bra HRR: X(a,b; f)
    def bra(a, b, f):
        nonlocal flops
        key = ("B", a, b, f)
        if key in names:
            return names[key]
        if sum(b) == 0:
            names[key] = src(a, f)
            return names[key]
        i = next(k for k in range(3) if b[k] > 0)
        b1 = sub(b, i)
        x = bra(add(a, i), b1, f)
        y = bra(a, b1, f)
        nm = f"h{len(lines)}"
        lines.append(f"const R {nm} = fma(AB{'xyz'[i]}, {y}, {x});")
        flops += 2
        names[key] = nm
        return nm

    def ket(a, b, c, d):
        nonlocal flops
        key = ("K", a, b, c, d)
        if key in names:
            return names[key]
        if sum(d) == 0:
            return bra(a, b, c)
        i = next(k for k in range(3) if d[k] > 0)
        d1 = sub(d, i)
        x = ket(a, b, add(c, i), d1)
        y = ket(a, b, c, d1)
        nm = f"h{len(lines)}"
        lines.append(f"const R {nm} = fma(CD{'xyz'[i]}, {y}, {x});")
        flops += 2
        names[key] = nm
        return nm

    outs = []
    for a in cart(la):
        for b in cart(lb):
            for c in cart(lc):
                for d in cart(ld):
                    f = comp_norm(a) * comp_norm(b) * comp_norm(c) * comp_norm(d)
                    v = ket(a, b, c, d)
                    if abs(f - 1.0) > 1e-15:
                        v = f"R({f!r}) * {v}"
                        flops += 1
                    outs.append(v)
    fn = f"hrr_{la}_{lb}_{lc}_{ld}"
    code = [
        f"// (ab|cd) block [{ncart(la)}][{ncart(lb)}][{ncart(lc)}][{ncart(ld)}] from {len(E)}x{nf} contracted [e0|f0]: {flops} flops",
        "template <typename R>",
        f"__device__ __forceinline__ void {fn}(const R* __restrict__ acc, const R ABx, const R ABy, const R ABz,",
        "    const R CDx, const R CDy, const R CDz, R* __restrict__ out) {",
    ] + ["  " + ln for ln in lines] + [f"  out[{k}] = {o};" for k, o in enumerate(outs)] + ["}", ""]
    return fn, len(E) * nf, flops, "\n".join(code)


def pair_classes():
    return [(a, b) for a in range(LMAX + 1) for b in range(a + 1)]


def quartet_classes():
    pcs = pair_classes()
    out = []
    for i, x in enumerate(pcs):
        for j, y in enumerate(pcs[: i + 1]):
            out.append(x + y)
    return out


def main(outdir):
    """Write eri_<tag>.h, fock_<tag>.hip per class, classes.h and eri_flops.json."""
    os.makedirs(outdir, exist_ok=True)
    table = {}
    classes = quartet_classes()
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        ev = (la, la + lb, lc, lc + ld)
        fn_v, nacc, fl_v, code_v = gen_vrr(*ev)
        fn_h, nacc_h, fl_h, code_h = gen_hrr(la, lb, lc, ld)
        assert nacc == nacc_h
        nout = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        struct = f"""struct Cls{tag} {{
  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld};
  static constexpr int NACC = {nacc}, NOUT = {nout};
  template <typename R>
  __device__ static __forceinline__ void vrr(const R* F, R PAx, R PAy, R PAz, R WPx, R WPy, R WPz,
      R QCx, R QCy, R QCz, R WQx, R WQy, R WQz, R oo2p, R oo2q, R oo2pq, R rho_p2, R rho_q2,
      R w, R* acc) {{
    {fn_v}<R>(F, PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz, oo2p, oo2q, oo2pq,
              rho_p2, rho_q2, w, acc);
  }}
  template <typename R>
  __device__ static __forceinline__ void hrr(const R* acc, R ABx, R ABy, R ABz, R CDx, R CDy,
                                             R CDz, R* out) {{
    {fn_h}<R>(acc, ABx, ABy, ABz, CDx, CDy, CDz, out);
  }}
}};
"""
        hdr = [f"// generated by gen_eri.py: class ({la}{lb}|{lc}{ld})", "#pragma once",
               "#include <hip/hip_runtime.h>", "namespace bscf {", "", code_v, code_h, struct,
               "}  // namespace bscf", ""]
        with open(os.path.join(outdir, f"eri_{tag}.h"), "w") as f:
            f.write("\n".join(hdr))
        tu = [f"// generated by gen_eri.py: kernels of class ({la}{lb}|{lc}{ld})",
              '#include "fock_kernel.h"', f'#include "eri_{tag}.h"', "namespace bscf {",
              f"void launch_fock_{tag}(const FockArgs& a, int fp32, hipStream_t s) {{",
              "  const int blocks = (a.nitems + 3) / 4;",
              "  if (blocks == 0) return;",
              (f"  if (fp32) hipLaunchKernelGGL((fock_kernel<Cls{tag}, float>), dim3(blocks), dim3(256), 0, s, a);\n  else"
               if la + lb + lc + ld < 7 else "  (void)fp32;  // rare heavy class: FP64 in every precision mode\n ") +
              f" hipLaunchKernelGGL((fock_kernel<Cls{tag}, double>), dim3(blocks), dim3(256), 0, s, a);",
              "}",
              f"void launch_tensor_{tag}(const TensorArgs& a, hipStream_t s) {{",
              "  if (a.nquart == 0) return;",
              f"  hipLaunchKernelGGL((tensor_kernel<Cls{tag}>), dim3((a.nquart + 63) / 64), dim3(64), 0, s, a);",
              "}"]
        if (la, lb) == (lc, ld):
            tu += [f"void launch_schwarz_{la}{lb}(const SchwarzArgs& a, hipStream_t s) {{",
                   "  if (a.npairs == 0) return;",
                   f"  hipLaunchKernelGGL((schwarz_kernel<Cls{tag}>), dim3((a.npairs + 255) / 256), dim3(256), 0, s, a);",
                   "}"]
        tu += ["}  // namespace bscf", ""]
        with open(os.path.join(outdir, f"fock_{tag}.hip"), "w") as f:
            f.write("\n".join(tu))
        table[tag] = dict(vrr_flops_per_prim=fl_v, hrr_flops=fl_h, nacc=nacc, ncart=nout)
    # registry
    reg = ["// generated by gen_eri.py: launcher registry", "#pragma once",
           '#include "fock_kernel.h"', "namespace bscf {"]
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        reg.append(f"void launch_fock_{tag}(const FockArgs&, int, hipStream_t);")
        reg.append(f"void launch_tensor_{tag}(const TensorArgs&, hipStream_t);")
    for (la, lb) in pair_classes():
        reg.append(f"void launch_schwarz_{la}{lb}(const SchwarzArgs&, hipStream_t);")
    reg.append(f"constexpr int kNumQuartetClasses = {len(classes)};")
    reg.append("struct QuartetClass { int la, lb, lc, ld; void (*fock)(const FockArgs&, int, hipStream_t);")
    reg.append("  void (*tensor)(const TensorArgs&, hipStream_t); double vrr_flops, hrr_flops; };")
    reg.append("inline const QuartetClass* quartet_classes() {")
    reg.append("  static const QuartetClass t[] = {")
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        reg.append(f"    {{{la}, {lb}, {lc}, {ld}, launch_fock_{tag}, launch_tensor_{tag}, "
                   f"{table[tag]['vrr_flops_per_prim']}.0, {table[tag]['hrr_flops']}.0}},")
    reg += ["  };", "  return t;", "}"]
    reg.append(f"constexpr int kNumPairClasses = {len(pair_classes())};")
    reg.append("inline void (*schwarz_launcher(int la, int lb))(const SchwarzArgs&, hipStream_t) {")
    for (la, lb) in pair_classes():
        reg.append(f"  if (la == {la} && lb == {lb}) return launch_schwarz_{la}{lb};")
    reg += ["  return nullptr;", "}", "}  // namespace bscf", ""]
    with open(os.path.join(outdir, "classes.h"), "w") as f:
        f.write("\n".join(reg))
    with open(os.path.join(outdir, "eri_flops.json"), "w") as f:
        json.dump(table, f, indent=1)
    return [f"{c[0]}{c[1]}{c[2]}{c[3]}" for c in classes]


if __name__ == "__main__":
    print(" ".join(main(sys.argv[1] if len(sys.argv) > 1 else "generated")))
