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
import re
import sys

LMAX = 2  # s, p, d


def write_if_changed(path, text):
    """Write only when the content differs (keeps mtimes for incremental builds)."""
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


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


def hrr_core(la, lb, lc, ld, src_name="acc", prefix="h", norm=True):
    """Straight-line HRR lines and the output expression of each (a,b,c,d)."""
    E = shells_range(la, la + lb)
    Fs = shells_range(lc, lc + ld)
    eidx = {e: k for k, e in enumerate(E)}
    fidx = {f: k for k, f in enumerate(Fs)}
    nf = len(Fs)
    lines = []
    flops = 0
    names = {}

    def src(e, f):
        return f"{src_name}[{eidx[e] * nf + fidx[f]}]"

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
        nm = f"{prefix}{len(lines)}"
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
        nm = f"{prefix}{len(lines)}"
        lines.append(f"const R {nm} = fma(CD{'xyz'[i]}, {y}, {x});")
        flops += 2
        names[key] = nm
        return nm

    outs = []
    for a in cart(la):
        for b in cart(lb):
            for c in cart(lc):
                for d in cart(ld):
                    v = ket(a, b, c, d)
                    if norm:
                        f = comp_norm(a) * comp_norm(b) * comp_norm(c) * comp_norm(d)
                        if abs(f - 1.0) > 1e-15:
                            v = f"R({f!r}) * {v}"
                            flops += 1
                    outs.append(((a, b, c, d), v))
    return lines, outs, flops, len(E) * nf


def gen_hrr(la, lb, lc, ld):
    """(ab|cd) from contracted [e0|f0], e in [la, la+lb], f in [lc, lc+ld]."""
    lines, outs, flops, nacc = hrr_core(la, lb, lc, ld)
    nf = len(shells_range(lc, lc + ld))
    fn = f"hrr_{la}_{lb}_{lc}_{ld}"
    code = [
        f"// (ab|cd) block [{ncart(la)}][{ncart(lb)}][{ncart(lc)}][{ncart(ld)}] from {nacc // nf}x{nf} contracted [e0|f0]: {flops} flops",
        "template <typename R>",
        f"__device__ __forceinline__ void {fn}(const R* __restrict__ acc, const R ABx, const R ABy, const R ABz,",
        "    const R CDx, const R CDy, const R CDz, R* __restrict__ out) {",
    ] + ["  " + ln for ln in lines] + [f"  out[{k}] = {o[1]};" for k, o in enumerate(outs)] + ["}", ""]
    return fn, nacc, flops, "\n".join(code)


def gen_grad(la, lb, lc, ld):
    """Gradient pieces of class (la lb|lc ld).

    VRR accumulates, per primitive quartet with weights w:
      RA = 2 alpha [e0|f0], e in [la+1, la+lb+1]   -> (a+1_i b|cd)
      RB = 2 beta  [e0|f0], e in [la, la+lb+1]     -> (a b+1_i|cd)
      RC = 2 gamma [e0|f0], f in [lc+1, lc+ld+1]   -> (ab|c+1_i d)
      LA, LB, LC = [e0|f0] on the lowered ranges   -> (a-1_i b|cd), ...
    and the contraction forms, with G the density factor per (a,b,c,d),
      gX_i = sum G (2 exp (x+1_i ..) - x_i (x-1_i ..))   for X = A, B, C.
    Classes with la+lb+lc+ld >= 6 contract every primitive quartet at once
    (no contracted accumulators) in three per-centre passes, each evaluating
    only the recurrence nodes its own sets need.
    """
    sets = [("RA", "wa", la + 1, la + lb + 1, lc, lc + ld),
            ("RB", "wb", la, la + lb + 1, lc, lc + ld),
            ("RC", "wc", la, la + lb, lc + 1, lc + ld + 1)]
    if la > 0:
        sets.append(("LA", None, la - 1, la - 1 + lb, lc, lc + ld))
    if lb > 0:
        sets.append(("LB", None, la, la + lb - 1, lc, lc + ld))
    if lc > 0:
        sets.append(("LC", None, la, la + lb, lc - 1, lc - 1 + ld))
    tag = f"{la}{lb}{lc}{ld}"
    sizes = {}
    targets = {}
    for nm, w, e0, e1, f0, f1 in sets:
        targets[nm] = [(e, f) for e in shells_range(e0, e1) for f in shells_range(f0, f1)]
        sizes[nm] = len(targets[nm])
    # contraction lines per set
    ca, cb, cc, cd = cart(la), cart(lb), cart(lc), cart(ld)
    gidx = {}
    k = 0
    for a in ca:
        for b in cb:
            for c in cc:
                for d in cd:
                    gidx[(a, b, c, d)] = k
                    k += 1
    nrm = {key: comp_norm(key[0]) * comp_norm(key[1]) * comp_norm(key[2]) * comp_norm(key[3])
           for key in gidx}
    hr = {"RA": (0, +1, (la + 1, lb, lc, ld)), "RB": (1, +1, (la, lb + 1, lc, ld)),
          "RC": (2, +1, (la, lb, lc + 1, ld)), "LA": (0, -1, (la - 1, lb, lc, ld)),
          "LB": (1, -1, (la, lb - 1, lc, ld)), "LC": (2, -1, (la, lb, lc - 1, ld))}
    con = {}
    cflops = 0
    for nm, *_ in sets:
        cen, sgn, cls = hr[nm]
        lines, outs, fl, _ = hrr_core(*cls, src_name=nm, prefix=f"{nm.lower()}_", norm=False)
        body = ["  " + ln for ln in lines]
        cflops += fl
        for comp, expr in outs:
            for i in range(3):
                t = list(comp)
                u = list(t[cen])
                if sgn > 0:
                    if u[i] == 0:
                        continue
                    u[i] -= 1
                    coef = 1.0
                else:
                    u[i] += 1
                    coef = -float(u[i])
                t[cen] = tuple(u)
                key = tuple(t)
                if key not in gidx:
                    continue
                c = coef * nrm[key]
                body.append(f"  g[{3 * cen + i}] = fma({c!r} * G[{gidx[key]}], double({expr}), g[{3 * cen + i}]);")
                cflops += 3
        con[nm] = body
    sig = ["template <typename R>",
           "__device__ {inl} void {fn}(const R* __restrict__ F, const R PAx, const R PAy, const R PAz,",
           "    const R WPx, const R WPy, const R WPz, const R QCx, const R QCy, const R QCz,",
           "    const R WQx, const R WQy, const R WQz, const R oo2p, const R oo2q, const R oo2pq,",
           "    const R rho_p2, const R rho_q2, const R wa, const R wb, const R wc{extra}) {{"]
    prim = la + lb + lc + ld >= 6
    flops = 0
    if not prim:
        v = VRR(0, 0, 0, 0)
        acc_lines = []
        for nm, w, *_ in sets:
            for kk, (e, f) in enumerate(targets[nm]):
                t = v.name(e, f, 0)
                acc_lines.append(f"  {nm}[{kk}] = fma({w or 'one'}, {t}, {nm}[{kk}]);")
                flops += 2
        flops += v.flops
        params = "".join(f", R* __restrict__ {s[0]}" for s in sets)
        code = [f"// gradient VRR of class ({tag}): {flops} flops per primitive quartet"]
        code += [s.format(inl="__forceinline__", fn=f"gvrr_{tag}", extra=params) for s in sig]
        code += ["  const R one = R(1);"] + ["  " + ln for ln in v.lines] + acc_lines + ["}", ""]
        code += [f"// gradient contraction of class ({tag}): {cflops} flops per quartet",
                 "template <typename R>",
                 f"__device__ __forceinline__ void gcon_{tag}({', '.join('const R* __restrict__ ' + s[0] for s in sets)},",
                 "    const R ABx, const R ABy, const R ABz, const R CDx, const R CDy, const R CDz,",
                 "    const double* __restrict__ G, double* __restrict__ g) {"]
        for nm, *_ in sets:
            code += con[nm]
        code += ["}", ""]
        # per-centre forms: the sets of one centre, with only the recurrence
        # nodes they need (used by classes whose six sets do not fit the lane's
        # registers; three passes over the primitives, one per centre)
        for X in "ABC":
            grp = [st for st in sets if st[0][1] == X]
            vx = VRR(0, 0, 0, 0)
            acc_x = []
            for nm, w, *_ in grp:
                for kk, (e, f) in enumerate(targets[nm]):
                    acc_x.append(f"  {nm}[{kk}] = fma({w or 'one'}, {vx.name(e, f, 0)}, {nm}[{kk}]);")
            px = "".join(f", R* __restrict__ {st[0]}" for st in grp)
            code += [f"// gradient VRR of class ({tag}), centre {X}"]
            code += [ln.format(inl="__forceinline__", fn=f"gvrr{X}_{tag}", extra=px) for ln in sig]
            code += ["  const R one = R(1);"] + ["  " + ln for ln in vx.lines] + acc_x + ["}", ""]
            code += [f"// gradient contraction of class ({tag}), centre {X}",
                     "template <typename R>",
                     f"__device__ __forceinline__ void gcon{X}_{tag}({', '.join('const R* __restrict__ ' + st[0] for st in grp)},",
                     "    const R ABx, const R ABy, const R ABz, const R CDx, const R CDy, const R CDz,",
                     "    const double* __restrict__ G, double* __restrict__ g) {"]
            for nm, *_ in grp:
                code += con[nm]
            code += ["}", ""]
        return sets, sizes, flops, cflops, "\n".join(code)
    code = []
    extra = (", const R ABx, const R ABy, const R ABz, const R CDx, const R CDy, const R CDz,"
             "\n    const double* __restrict__ G, double* __restrict__ g")
    for X in "ABC":
        grp = [s for s in sets if s[0][1] == X]
        v = VRR(0, 0, 0, 0)
        asg = []
        for nm, w, *_ in grp:
            asg.append(f"  R {nm}[{sizes[nm]}];")
            for kk, (e, f) in enumerate(targets[nm]):
                t = v.name(e, f, 0)
                asg.append(f"  {nm}[{kk}] = {w or 'one'} * {t};")
        flops += v.flops
        code += [f"// gradient of class ({tag}), centre {X}, one primitive quartet"]
        code += [s.format(inl="__noinline__", fn=f"gprim{X}_{tag}", extra=extra) for s in sig]
        code += ["  const R one = R(1);"] + ["  " + ln for ln in v.lines] + asg
        for nm, *_ in grp:
            code += con[nm]
        code += ["}", ""]
    code += ["template <typename R>",
             f"__device__ __forceinline__ void gprim_{tag}(const R* __restrict__ F, const R PAx, const R PAy, const R PAz,",
             "    const R WPx, const R WPy, const R WPz, const R QCx, const R QCy, const R QCz,",
             "    const R WQx, const R WQy, const R WQz, const R oo2p, const R oo2q, const R oo2pq,",
             "    const R rho_p2, const R rho_q2, const R wa, const R wb, const R wc,",
             "    const R ABx, const R ABy, const R ABz, const R CDx, const R CDy, const R CDz,",
             "    const double* __restrict__ G, double* __restrict__ g) {"]
    for X in "ABC":
        code.append(f"  gprim{X}_{tag}<R>(F, PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz,"
                    " oo2p, oo2q, oo2pq, rho_p2, rho_q2, wa, wb, wc, ABx, ABy, ABz, CDx, CDy, CDz, G, g);")
    code += ["}", ""]
    return sets, sizes, flops, cflops, "\n".join(code)


def pair_classes():
    return [(a, b) for a in range(LMAX + 1) for b in range(a + 1)]


def quartet_classes():
    pcs = pair_classes()
    out = []
    for i, x in enumerate(pcs):
        for j, y in enumerate(pcs[: i + 1]):
            out.append(x + y)
    return out


LANE_E_MAX = 5   # one-lane-per-quartet Fock kernels up to this total L
LANE_G_MAX = 5   # one-lane-per-quartet gradient kernels up to this total L
SPLIT_GRAD_ACC = 120   # lane gradient classes with more accumulators run one pass per centre
SUB_GRAD_ACC = 128     # ... and split each centre's pass into parts of at most this many


def coop_tu(la, lb, lc, ld):
    """Cooperative kernels of one class: node tables, traits, launchers."""
    import gen_coop
    tag = f"{la}{lb}{lc}{ld}"
    pe = gen_coop.energy_program(la, lb, lc, ld)
    pg = gen_coop.grad_program(la, lb, lc, ld)

    def traits(name, p, prefix, grad):
        acc = [f"  __device__ static const {t}* {f}() {{ return {prefix}_{f}; }}"
               for t, f in [("int", "vrr_lstart"), ("unsigned long long", "vrr_node"),
                            ("unsigned int", "vrr_term"), ("int", "hrr_lstart"),
                            ("unsigned long long", "hrr_node"), ("unsigned int", "hrr_term"),
                            ("unsigned short", "acc_slot"), ("unsigned short", "tgt_slot"),
                            ("unsigned char", "tgt_w")]]
        if grad:
            acc += [f"  __device__ static const {t}* {f}() {{ return {prefix}_{f}; }}"
                    for t, f in [("int", "con_lstart"), ("unsigned long long", "con_word"),
                                 ("double", "con_ctab")]]
            extra = (f", NCLEV = {len(p['con_lstart']) - 1}, NCTAB = {len(set(p['con_c']))}"
                     f";\n  static constexpr int QB = {gen_coop.grad_quartets_per_block(p)}, "
                     f"NTQ = {gen_coop.grad_block_threads(p)};   // quartets and threads per block")
        else:
            acc += [f"  __device__ static const {t}* {f}() {{ return {prefix}_{f}; }}"
                    for t, f in [("unsigned short", "out_slot"), ("double", "norm")]]
            extra = ""
        return "\n".join([
            f"struct {name} {{",
            f"  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld}, L = {p['L']};",
            f"  static constexpr int NSLOT = {p['nslot']}, NACC = {p['nacc']}, NOUT = {p['nout']}, "
            f"FSLOT = {p['fslot']};",
            f"  static constexpr int NVLEV = {len(p['vrr'][0]) - 1}, NHLEV = {len(p['hrr'][0]) - 1}{extra};",
            f"  static constexpr int NT = {gen_coop.threads_per_block(p, grad)};   // threads per quartet",
        ] + acc + ["};", ""])

    lines = [f"// generated by gen_eri.py / gen_coop.py: cooperative kernels of class ({la}{lb}|{lc}{ld})",
             '#include "coop_kernel.h"', "namespace bscf {", "namespace {",
             gen_coop.emit_tables(f"cE{tag}", pe), gen_coop.emit_tables(f"cG{tag}", pg, grad=True),
             traits(f"CoopE{tag}", pe, f"cE{tag}", False), traits(f"CoopG{tag}", pg, f"cG{tag}", True),
             "}  // namespace",
             f"void launch_coop_fock_{tag}(const FockArgs& a, hipStream_t s) {{",
             "  if (a.nitems == 0) return;",
             f"  hipLaunchKernelGGL((coop_fock_kernel<CoopE{tag}>), dim3(coop_blocks(a.nitems)), dim3(CoopE{tag}::NT), 0, s, a);",
             "}",
             f"void launch_coop_grad_{tag}(const GradArgs& a, hipStream_t s) {{",
             "  if (a.nitems == 0) return;",
             f"  hipLaunchKernelGGL((coop_grad_kernel<CoopG{tag}>), dim3(coop_blocks_q(a.nitems, CoopG{tag}::QB)), dim3(CoopG{tag}::NTQ), 0, s, a);",
             "}",
             f"void launch_coop_tensor_{tag}(const TensorArgs& a, hipStream_t s) {{",
             "  if (a.nquart == 0) return;",
             f"  hipLaunchKernelGGL((coop_tensor_kernel<CoopE{tag}>), dim3(a.nquart), dim3(CoopE{tag}::NT), 0, s, a);",
             "}",
             f"int coop_private_bytes_{tag}(int which) {{",
             "  hipFuncAttributes at{};",
             f"  const void* f = which ? reinterpret_cast<const void*>(&coop_grad_kernel<CoopG{tag}>)",
             f"                        : reinterpret_cast<const void*>(&coop_fock_kernel<CoopE{tag}>);",
             "  if (hipFuncGetAttributes(&at, f) != hipSuccess) return -1;",
             "  return (int)at.localSizeBytes;",
             "}"]
    if (la, lb) == (lc, ld):
        lines += [f"void launch_coop_schwarz_{la}{lb}(const SchwarzArgs& a, hipStream_t s) {{",
                  "  if (a.npairs == 0) return;",
                  f"  hipLaunchKernelGGL((coop_schwarz_kernel<CoopE{tag}>), dim3(a.npairs), dim3(CoopE{tag}::NT), 0, s, a);",
                  "}"]
    lines += ["}  // namespace bscf", ""]
    return "\n".join(lines), pe, pg


def prim_flops(L):
    """FLOPs of one primitive quartet outside the VRR, counted from the lane
    kernel's primitive loop (eri_block_body in fock_kernel.h) and from
    boys_f64 (boys.h); an FMA counts two, a reciprocal square root one.

    Setup (every class):
      p + q 1; rsqrt(p + q) 1; 1/(p + q) as its square 1; rho = p q/(p + q) 2;
      PQ 3; T = rho |PQ|^2 6; prefactor C_ab C_cd rsqrt(p + q) 2      -> 16
    Setup of the VRR arguments (L > 0):
      q/(p + q), p/(p + q) 2; -q/(p + q) PQ and p/(p + q) PQ 6;
      1/(2(p + q)) 1; the two 1/(2p) q/(p + q) factors 2                -> 11
    Boys function below T = 40 (the branch every integral of these systems
    takes, T being far smaller):
      grid index T/0.1 1; d = T - 0.1 k 2; 8-term Taylor of F_L, 7 x (mul +
      FMA) 21; F_L scaled 1                                             -> 25
      L > 0: exp(-T) from the 9-term Taylor of exp, 8 x (mul + FMA), times
      the table's exp(-T_k) 25; 2T 1; per m < L FMA, 1/(2m+1) and the
      scaling 4                                                         -> 26 + 4L
    L = 0 adds acc += F_0 (1) and runs no VRR."""
    f = 16 + 25
    if L == 0:
        return f + 1
    return f + 11 + 26 + 4 * L


def main(outdir):
    """Write the per-class headers and translation units, classes.h and
    eri_flops.json."""
    os.makedirs(outdir, exist_ok=True)
    table = {}
    classes = quartet_classes()
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        L = la + lb + lc + ld
        ev = (la, la + lb, lc, lc + ld)
        fn_v, nacc, fl_v, code_v = gen_vrr(*ev)
        fn_h, nacc_h, fl_h, code_h = gen_hrr(la, lb, lc, ld)
        assert nacc == nacc_h
        nout = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        # per primitive quartet in all: setup, Boys and (L > 0) the VRR
        table[tag] = dict(vrr_flops_per_prim=fl_v, hrr_flops=fl_h, nacc=nacc, ncart=nout,
                          prim_flops=prim_flops(L) + (fl_v if L > 0 else 0))
        if L <= LANE_E_MAX:
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
            write_if_changed(os.path.join(outdir, f"eri_{tag}.h"), "\n".join(hdr))
            tu = [f"// generated by gen_eri.py: kernels of class ({la}{lb}|{lc}{ld})",
                  '#include "fock_kernel.h"', f'#include "eri_{tag}.h"', "namespace bscf {",
                  f"// mode 0: FP64; 1: FP32; 2: mixed (each row's FP64 prefix in FP64, the rest in FP32)",
                  f"void launch_fock_{tag}(const FockArgs& a, int mode, hipStream_t s) {{",
                  "  if (a.nunits == 0) return;",
                  f"  const size_t lds = sizeof(double) * unit_lds_doubles({la}, {lb}, a.nmax, a.max_prims);",
                  f"  if (mode == 2) hipLaunchKernelGGL((fock_unit_kernel<Cls{tag}, double, true>), dim3(a.nunits), dim3(a.unit_threads), lds, s, a);",
                  f"  else if (mode == 1) hipLaunchKernelGGL((fock_unit_kernel<Cls{tag}, float>), dim3(a.nunits), dim3(a.unit_threads), lds, s, a);",
                  f"  else hipLaunchKernelGGL((fock_unit_kernel<Cls{tag}, double>), dim3(a.nunits), dim3(a.unit_threads), lds, s, a);",
                  "}",
                  f"int fock_private_bytes_{tag}(int mode) {{",
                  "  hipFuncAttributes at{};",
                  f"  const void* f = mode == 2 ? reinterpret_cast<const void*>(&fock_unit_kernel<Cls{tag}, double, true>)",
                  f"                : mode == 1 ? reinterpret_cast<const void*>(&fock_unit_kernel<Cls{tag}, float>)",
                  f"                            : reinterpret_cast<const void*>(&fock_unit_kernel<Cls{tag}, double>);",
                  "  if (hipFuncGetAttributes(&at, f) != hipSuccess) return -1;",
                  "  return (int)at.localSizeBytes;",
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
            write_if_changed(os.path.join(outdir, f"fock_{tag}.hip"), "\n".join(tu))
        ctu, pe, pg = coop_tu(la, lb, lc, ld)
        write_if_changed(os.path.join(outdir, f"coop_{tag}.hip"), ctu)
        table[tag]["coop_lds_bytes"] = [8 * pe["nslot"], 8 * (pg["nslot"] + nout)]
    # gradient classes (lane form)
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        sets, sizes, gfl, cfl, code = gen_grad(la, lb, lc, ld)
        table[tag]["grad_vrr_flops_per_prim"] = gfl
        # per primitive quartet in all: setup and Boys to L + 1, the raised and lowered VRR
        table[tag]["grad_prim_flops"] = prim_flops(la + lb + lc + ld + 1) + gfl
        table[tag]["grad_contract_flops"] = cfl
        if la + lb + lc + ld > LANE_G_MAX:
            continue
        names = [s[0] for s in sets]
        allsets = ["RA", "RB", "RC", "LA", "LB", "LC"]
        szs = ", ".join(f"N{s} = {sizes.get(s, 1)}" for s in allsets)
        arg = ", ".join(s for s in names)
        split = sum(sizes.values()) > SPLIT_GRAD_ACC
        per_pass = max(sizes.get(f"R{X}", 0) + sizes.get(f"L{X}", 0) for X in "ABC")
        nsub = -(-per_pass // SUB_GRAD_ACC) if split else 1
        def cargs(X):   # the per-centre functions' set arguments: S1 = raised, S2 = lowered
            return "S1" + (", S2" if f"L{X}" in names else "")
        vx = "\n".join(
            f"    {'if' if k == 0 else 'else if'} constexpr (X == {k}) gvrr{X}_{tag}<R>(F, PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz, oo2p, oo2q, oo2pq, rho_p2, rho_q2, wa, wb, wc, {cargs(X)});"
            for k, X in enumerate("ABC"))
        cx = "\n".join(
            f"    {'if' if k == 0 else 'else if'} constexpr (X == {k}) gcon{X}_{tag}<R>({cargs(X)}, ABx, ABy, ABz, CDx, CDy, CDz, G, g);"
            for k, X in enumerate("ABC"))
        wrap = f"""struct ClsG{tag} {{
  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld};
  static constexpr bool PRIM = false;
  static constexpr bool SPLIT = {'true' if split else 'false'};   // one pass per centre
  static constexpr int NSUB = {nsub};   // sub-passes per centre pass
  static constexpr int {szs};
  // centre X (0 = A, 1 = B, 2 = C): S1 = its raised set, S2 = its lowered set (if any)
  template <int X, typename R>
  __device__ static __forceinline__ void vrrx(const R* F, R PAx, R PAy, R PAz, R WPx, R WPy, R WPz,
      R QCx, R QCy, R QCz, R WQx, R WQy, R WQz, R oo2p, R oo2q, R oo2pq, R rho_p2, R rho_q2,
      R wa, R wb, R wc, R* S1, R* S2) {{
    (void)S2;
{vx}
  }}
  template <int X, typename R>
  __device__ static __forceinline__ void conx(const R* S1, const R* S2, R ABx, R ABy, R ABz,
      R CDx, R CDy, R CDz, const double* G, double* g) {{
    (void)S2;
{cx}
  }}
  template <typename R>
  __device__ static __forceinline__ void vrr(const R* F, R PAx, R PAy, R PAz, R WPx, R WPy, R WPz,
      R QCx, R QCy, R QCz, R WQx, R WQy, R WQz, R oo2p, R oo2q, R oo2pq, R rho_p2, R rho_q2,
      R wa, R wb, R wc, R* RA, R* RB, R* RC, R* LA, R* LB, R* LC) {{
    gvrr_{tag}<R>(F, PAx, PAy, PAz, WPx, WPy, WPz, QCx, QCy, QCz, WQx, WQy, WQz, oo2p, oo2q,
                  oo2pq, rho_p2, rho_q2, wa, wb, wc, {arg});
  }}
  template <typename R>
  __device__ static __forceinline__ void con(const R* RA, const R* RB, const R* RC, const R* LA,
      const R* LB, const R* LC, R ABx, R ABy, R ABz, R CDx, R CDy, R CDz, const double* G,
      double* g) {{
    gcon_{tag}<R>({arg}, ABx, ABy, ABz, CDx, CDy, CDz, G, g);
  }}
}};
"""
        hdr = [f"// generated by gen_eri.py: gradient of class ({la}{lb}|{lc}{ld})", "#pragma once",
               "#include <hip/hip_runtime.h>", "namespace bscf {", "", code, wrap,
               "}  // namespace bscf", ""]
        write_if_changed(os.path.join(outdir, f"grad_{tag}.h"), "\n".join(hdr))
        tu = [f"// generated by gen_eri.py: gradient kernel of class ({la}{lb}|{lc}{ld})",
              '#include "grad_kernel.h"', f'#include "grad_{tag}.h"', "namespace bscf {",
              f"void launch_grad_{tag}(const GradArgs& a, hipStream_t s) {{",
              "  if (a.nunits == 0) return;",
              f"  const size_t lds = sizeof(double) * grad_unit_lds_doubles({la}, {lb}, a.nmax, a.max_atoms, a.max_prims);",
              f"  hipLaunchKernelGGL((grad_unit_kernel<ClsG{tag}>), dim3(a.nunits), dim3(a.unit_threads), lds, s, a);",
              "}",
              f"int grad_private_bytes_{tag}() {{",
              "  hipFuncAttributes at{};",
              f"  if (hipFuncGetAttributes(&at, reinterpret_cast<const void*>(&grad_unit_kernel<ClsG{tag}>)) != hipSuccess) return -1;",
              "  return (int)at.localSizeBytes;",
              "}", "}  // namespace bscf", ""]
        write_if_changed(os.path.join(outdir, f"grad_{tag}.hip"), "\n".join(tu))
    # drop translation units of an earlier configuration
    for fn in os.listdir(outdir):
        m = re.match(r"(fock|grad|eri)_(\d{4})\.(hip|h)$", fn)
        if not m:
            continue
        Lx = sum(int(ch) for ch in m.group(2))
        lim = LANE_G_MAX if m.group(1) == "grad" else LANE_E_MAX
        if Lx > lim:
            os.remove(os.path.join(outdir, fn))
    # registry
    reg = ["// generated by gen_eri.py: launcher registry", "#pragma once",
           '#include "fock_kernel.h"', '#include "grad.h"', "namespace bscf {"]
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        L = la + lb + lc + ld
        if L <= LANE_E_MAX:
            reg.append(f"void launch_fock_{tag}(const FockArgs&, int, hipStream_t);")
            reg.append(f"int fock_private_bytes_{tag}(int);")
            reg.append(f"void launch_tensor_{tag}(const TensorArgs&, hipStream_t);")
        if L <= LANE_G_MAX:
            reg.append(f"void launch_grad_{tag}(const GradArgs&, hipStream_t);")
            reg.append(f"int grad_private_bytes_{tag}();")
        reg.append(f"void launch_coop_fock_{tag}(const FockArgs&, hipStream_t);")
        reg.append(f"void launch_coop_grad_{tag}(const GradArgs&, hipStream_t);")
        reg.append(f"void launch_coop_tensor_{tag}(const TensorArgs&, hipStream_t);")
        reg.append(f"int coop_private_bytes_{tag}(int);")
    for (la, lb) in pair_classes():
        if 2 * (la + lb) <= LANE_E_MAX:
            reg.append(f"void launch_schwarz_{la}{lb}(const SchwarzArgs&, hipStream_t);")
        else:
            reg.append(f"void launch_coop_schwarz_{la}{lb}(const SchwarzArgs&, hipStream_t);")
    reg.append(f"constexpr int kNumQuartetClasses = {len(classes)};")
    reg += ["// lane: one quartet per lane (nullptr where not generated); coop: one per wavefront",
            "struct QuartetClass {",
            "  int la, lb, lc, ld;",
            "  void (*fock)(const FockArgs&, int, hipStream_t);",
            "  void (*coop_fock)(const FockArgs&, hipStream_t);",
            "  void (*grad)(const GradArgs&, hipStream_t);",
            "  void (*coop_grad)(const GradArgs&, hipStream_t);",
            "  void (*tensor)(const TensorArgs&, hipStream_t);",
            "  // FLOPs per primitive quartet (setup, Boys, VRR) and per contracted quartet (HRR),",
            "  // of the Fock build and of the gradient (its contraction with the density factors)",
            "  double prim_flops, hrr_flops, grad_prim_flops, grad_con_flops;",
            "  int (*fock_private_bytes)(int);",
            "  int (*grad_private_bytes)();",
            "  int (*coop_private_bytes)(int);",
            "};",
            "inline const QuartetClass* quartet_classes() {",
            "  static const QuartetClass t[] = {"]
    for (la, lb, lc, ld) in classes:
        tag = f"{la}{lb}{lc}{ld}"
        L = la + lb + lc + ld
        le, lg = L <= LANE_E_MAX, L <= LANE_G_MAX
        t = table[tag]
        reg.append(f"    {{{la}, {lb}, {lc}, {ld}, {f'launch_fock_{tag}' if le else 'nullptr'}, "
                   f"launch_coop_fock_{tag}, {f'launch_grad_{tag}' if lg else 'nullptr'}, "
                   f"launch_coop_grad_{tag}, {f'launch_tensor_{tag}' if le else f'launch_coop_tensor_{tag}'}, "
                   f"{t['prim_flops']}.0, {t['hrr_flops']}.0, {t['grad_prim_flops']}.0, "
                   f"{t['grad_contract_flops']}.0, {f'fock_private_bytes_{tag}' if le else 'nullptr'}, "
                   f"{f'grad_private_bytes_{tag}' if lg else 'nullptr'}, coop_private_bytes_{tag}}},")
    reg += ["  };", "  return t;", "}"]
    reg.append(f"constexpr int kNumPairClasses = {len(pair_classes())};")
    reg.append("inline void (*schwarz_launcher(int la, int lb))(const SchwarzArgs&, hipStream_t) {")
    for (la, lb) in pair_classes():
        fn = f"launch_schwarz_{la}{lb}" if 2 * (la + lb) <= LANE_E_MAX else f"launch_coop_schwarz_{la}{lb}"
        reg.append(f"  if (la == {la} && lb == {lb}) return {fn};")
    reg += ["  return nullptr;", "}", "}  // namespace bscf", ""]
    write_if_changed(os.path.join(outdir, "classes.h"), "\n".join(reg))
    write_if_changed(os.path.join(outdir, "eri_flops.json"), json.dumps(table, indent=1))
    return [f"{c[0]}{c[1]}{c[2]}{c[3]}" for c in classes]


if __name__ == "__main__":
    print(" ".join(main(sys.argv[1] if len(sys.argv) > 1 else "generated")))
