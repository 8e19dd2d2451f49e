#!/usr/bin/env python3
"""Node tables for the cooperative (one wavefront per shell quartet) kernels.

For classes of high angular momentum the straight-line, one-lane-per-quartet
code spills most of its state; instead the recurrence graph of one quartet is
evaluated by all 64 lanes of a wavefront level by level out of LDS.  This
module builds that graph from the same recurrences as gen_eri.py:

  * Obara-Saika VRR nodes [e0|f0]^(m) (bra and ket steps, see gen_eri.py),
    evaluated for every primitive quartet and accumulated into contracted
    targets (weighted by 2 alpha, 2 beta, 2 gamma for the gradient sets);
  * Head-Gordon-Pople HRR nodes on the contracted targets;
  * for the gradient, the contraction terms g_k += c * G[idx] * value.

Every node is dst = sum_t mult_t * scalar[sel_t] * slot[src_t]; nodes are
grouped into levels (inputs only from earlier levels) and LDS slots are reused
once a value's last reader level has completed.  Scalar selectors:
"""

from __future__ import annotations

from gen_eri import cart, ncart, shells_range, sub, add, comp_norm

SEL = {"one": 0, "PAx": 1, "PAy": 2, "PAz": 3, "WPx": 4, "WPy": 5, "WPz": 6,
       "QCx": 7, "QCy": 8, "QCz": 9, "WQx": 10, "WQy": 11, "WQz": 12,
       "oo2p": 13, "oo2q": 14, "oo2pq": 15, "rho_p2": 16, "rho_q2": 17,
       "ABx": 18, "ABy": 19, "ABz": 20, "CDx": 21, "CDy": 22, "CDz": 23,
       "wa": 24, "wb": 25, "wc": 26}
NSEL = 27
XYZ = "xyz"


class Graph:
    """Nodes keyed by a hashable key; node = list of (sel, mult, src key)."""

    def __init__(self):
        self.nodes = {}        # key -> terms
        self.order = []        # insertion order (topological)

    def add(self, key, terms):
        if key not in self.nodes:
            self.nodes[key] = terms
            self.order.append(key)
        return key


def vrr_graph(targets, L):
    """VRR nodes needed for targets [(e, f)] at m = 0; inputs ("F", m)."""
    g = Graph()

    def node(e, f, m):
        if min(e) < 0 or min(f) < 0:
            return None
        key = ("V", e, f, m)
        if key in g.nodes:
            return key
        if sum(e) == 0 and sum(f) == 0:
            return ("F", m)
        terms = []
        if sum(f) > 0:
            i = next(k for k in range(3) if f[k] > 0)
            f1 = sub(f, i)
            terms.append(("QC" + XYZ[i], 1.0, node(e, f1, m)))
            terms.append(("WQ" + XYZ[i], 1.0, node(e, f1, m + 1)))
            if f1[i] > 0:
                f2 = sub(f1, i)
                terms.append(("oo2q", float(f1[i]), node(e, f2, m)))
                terms.append(("rho_q2", -float(f1[i]), node(e, f2, m + 1)))
            if e[i] > 0:
                terms.append(("oo2pq", float(e[i]), node(sub(e, i), f1, m + 1)))
        else:
            i = next(k for k in range(3) if e[k] > 0)
            e1 = sub(e, i)
            terms.append(("PA" + XYZ[i], 1.0, node(e1, f, m)))
            terms.append(("WP" + XYZ[i], 1.0, node(e1, f, m + 1)))
            if e1[i] > 0:
                e2 = sub(e1, i)
                terms.append(("oo2p", float(e1[i]), node(e2, f, m)))
                terms.append(("rho_p2", -float(e1[i]), node(e2, f, m + 1)))
        terms = [t for t in terms if t[2] is not None]
        return g.add(key, terms)

    out = [node(e, f, 0) for e, f in targets]
    return g, out


def hrr_graph(g, la, lb, lc, ld, src, tag):
    """HRR nodes on contracted inputs src(e, f) -> key; returns output keys
    in (a, b, c, d) lexicographic order.  `tag` names the input set."""
    tag = (la, lb, lc, ld, tag)

    def bra(a, b, f):
        if sum(b) == 0:
            return src(a, f)
        key = ("B", tag, a, b, f)
        if key in g.nodes:
            return key
        i = next(k for k in range(3) if b[k] > 0)
        b1 = sub(b, i)
        return g.add(key, [("one", 1.0, bra(add(a, i), b1, f)), ("AB" + XYZ[i], 1.0, bra(a, b1, f))])

    def ket(a, b, c, d):
        if sum(d) == 0:
            return bra(a, b, c)
        key = ("K", tag, a, b, c, d)
        if key in g.nodes:
            return key
        i = next(k for k in range(3) if d[k] > 0)
        d1 = sub(d, i)
        return g.add(key, [("one", 1.0, ket(a, b, add(c, i), d1)), ("CD" + XYZ[i], 1.0, ket(a, b, c, d1))])

    return [ket(a, b, c, d) for a in cart(la) for b in cart(lb) for c in cart(lc) for d in cart(ld)]


def levels_of(g, inputs):
    lev = {k: 0 for k in inputs}
    for k in g.order:
        lev[k] = 1 + max(lev[t[2]] for t in g.nodes[k])
    return lev


def schedule(g, inputs, fixed, outputs, first_free, uses=None, lev=None):
    """Assign slots to the nodes of g (inputs already in `fixed`).  Values are
    freed after the level of their last reader (node, or an extra use given in
    `uses` as key -> level); `outputs` stay live.  `lev` may give the levels.
    Returns (levels: list of node lists, slot map, number of slots)."""
    if lev is None:
        lev = levels_of(g, inputs)
    nlev = max([lev[k] for k in g.order], default=0)
    by_level = [[] for _ in range(nlev + 1)]
    for k in g.order:
        by_level[lev[k]].append(k)
    last = {}
    for k in g.order:
        for t in g.nodes[k]:
            last[t[2]] = max(last.get(t[2], 0), lev[k])
    for k, l in (uses or {}).items():
        last[k] = max(last.get(k, 0), l)
    keep = set(outputs)
    slot = dict(fixed)
    free = []
    top = first_free
    release_at = {}
    for k in inputs:
        if k not in keep and k in last:
            release_at.setdefault(last[k], []).append(slot[k])
    free.extend(release_at.pop(0, []))
    for L in range(1, nlev + 1):
        for k in by_level[L]:
            if free:
                slot[k] = free.pop()
            else:
                slot[k] = top
                top += 1
            if k not in keep:
                if k in last:
                    release_at.setdefault(last[k], []).append(slot[k])
                else:
                    release_at.setdefault(L, []).append(slot[k])
        free.extend(release_at.pop(L, []))
    return by_level[1:], slot, top


def encode(levels, slot):
    """Flatten levels into (level_start[], node_dst[], node_t0[], term_src[],
    term_sel[], term_mult[])."""
    lstart, dst, t0, src, sel, mult = [0], [], [], [], [], []
    for lv in levels:
        for k, terms in lv:
            dst.append(slot[k])
            t0.append(len(src))
            for s, m, x in terms:
                src.append(slot[x])
                sel.append(SEL[s])
                mult.append(m)
        lstart.append(len(dst))
    t0.append(len(src))
    return lstart, dst, t0, src, sel, mult


def energy_program(la, lb, lc, ld):
    """Tables of the cooperative Fock-build evaluator of class (la lb|lc ld).

    Slots: NACC contracted accumulators at 0.., then F_m, then VRR
    temporaries; after the primitive loop the HRR temporaries and outputs
    reuse everything above the accumulators (and the accumulators once read)."""
    L = la + lb + lc + ld
    targets = [(e, f) for e in shells_range(la, la + lb) for f in shells_range(lc, lc + ld)]
    gv, tkeys = vrr_graph(targets, L)
    nacc = len(targets)
    acc0 = 0
    acc_slot = [acc0 + k for k in range(nacc)]
    inputs = [("F", m) for m in range(L + 1)]
    fixed = {k: nacc + m for m, k in enumerate(inputs)}
    lv_v, slot_v, top_v = schedule(gv, inputs, fixed, set(tkeys), nacc + L + 1)
    # a target may be an input F_m itself (only for L = 0 classes)
    tgt_slot = [slot_v[k] for k in tkeys]
    # HRR on accumulators
    gh = Graph()
    amap = {("A", e, f): acc0 + k for k, (e, f) in enumerate(targets)}
    outs = hrr_graph(gh, la, lb, lc, ld, lambda e, f: ("A", e, f), "A")
    lv_h, slot_h, top_h = schedule(gh, list(amap), amap, set(outs), nacc)
    out_slot = [slot_h[k] for k in outs]
    assert len(set(out_slot)) == len(out_slot)   # outputs are scaled in place
    norms = [comp_norm(a) * comp_norm(b) * comp_norm(c) * comp_norm(d)
             for a in cart(la) for b in cart(lb) for c in cart(lc) for d in cart(ld)]
    vrr = encode([[(k, gv.nodes[k]) for k in lv] for lv in lv_v], slot_v)
    hrr = encode([[(k, gh.nodes[k]) for k in lv] for lv in lv_h], slot_h)
    return dict(L=L, lsh=(la, lb, lc, ld), nslot=max(top_h, top_v), vrr=vrr, hrr=hrr, acc_slot=acc_slot,
                tgt_slot=tgt_slot, tgt_w=[0] * nacc, out_slot=out_slot, norms=norms,
                nacc=nacc, nout=len(outs), fslot=nacc)


def grad_program(la, lb, lc, ld):
    """Tables of the cooperative gradient evaluator of class (la lb|lc ld).

    Per primitive quartet the VRR feeds the weighted sets RA, RB, RC (2 alpha,
    2 beta, 2 gamma) and the lowered sets LA, LB, LC; after the primitive loop
    the HRR of every set is contracted with G into g[0..8] (A, B, C centres).
    """
    L = la + lb + lc + ld + 1
    sets = [("RA", "wa", la + 1, la + lb + 1, lc, lc + ld, 0, +1, (la + 1, lb, lc, ld)),
            ("RB", "wb", la, la + lb + 1, lc, lc + ld, 1, +1, (la, lb + 1, lc, ld)),
            ("RC", "wc", la, la + lb, lc + 1, lc + ld + 1, 2, +1, (la, lb, lc + 1, ld))]
    if la > 0:
        sets.append(("LA", "one", la - 1, la - 1 + lb, lc, lc + ld, 0, -1, (la - 1, lb, lc, ld)))
    if lb > 0:
        sets.append(("LB", "one", la, la + lb - 1, lc, lc + ld, 1, -1, (la, lb - 1, lc, ld)))
    if lc > 0:
        sets.append(("LC", "one", la, la + lb, lc - 1, lc - 1 + ld, 2, -1, (la, lb, lc - 1, ld)))
    targets, tw, tset = [], [], []
    for nm, w, e0, e1, f0, f1, *_ in sets:
        for e in shells_range(e0, e1):
            for f in shells_range(f0, f1):
                targets.append((e, f))
                tw.append(SEL[w])
                tset.append(nm)
    gv, tkeys = vrr_graph(sorted(set(targets)), L)
    key_of = dict(zip(sorted(set(targets)), tkeys))
    nacc = len(targets)
    acc0 = 0
    acc_slot = [acc0 + k for k in range(nacc)]
    inputs = [("F", m) for m in range(L + 1)]
    fixed = {k: nacc + m for m, k in enumerate(inputs)}
    lv_v, slot_v, top_v = schedule(gv, inputs, fixed, set(tkeys), nacc + L + 1)
    tgt_slot = [slot_v[key_of[t]] for t in targets]
    # HRR of each set on its accumulators, then contraction terms
    gh = Graph()
    amap = {}
    k = 0
    for nm, w, e0, e1, f0, f1, *_ in sets:
        for e in shells_range(e0, e1):
            for f in shells_range(f0, f1):
                amap[(nm, e, f)] = acc0 + k
                k += 1
    gidx = {}
    n = 0
    for a in cart(la):
        for b in cart(lb):
            for c in cart(lc):
                for d in cart(ld):
                    gidx[(a, b, c, d)] = n
                    n += 1
    nrm = {key: comp_norm(key[0]) * comp_norm(key[1]) * comp_norm(key[2]) * comp_norm(key[3])
           for key in gidx}
    con = []   # (value key, g component, G index, coefficient)
    for nm, w, e0, e1, f0, f1, cen, sgn, cls in sets:
        outs = hrr_graph(gh, *cls, lambda e, f, nm=nm: (nm, e, f), nm)
        comps = [(a, b, c, d) for a in cart(cls[0]) for b in cart(cls[1])
                 for c in cart(cls[2]) for d in cart(cls[3])]
        for key, comp in zip(outs, comps):
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
                kk = tuple(t)
                if kk in gidx:
                    con.append((key, 3 * cen + i, gidx[kk], coef * nrm[kk]))
    # sets are transformed one after another (their levels offset), every value
    # is contracted right after the level that produced it (the set's first
    # level: accumulators used directly) and its slot is freed after that level
    base_lev = levels_of(gh, list(amap))
    hlev, base = {}, 0
    for nm, *_ in sets:
        mine = [k for k in gh.order if k[1][4] == nm]
        top = max([base_lev[k] for k in mine], default=0)
        for k in mine:
            hlev[k] = base + base_lev[k]
        for k in amap:
            if k[0] == nm:
                hlev[k] = base
        base += top + 1
    uses = {c[0]: hlev[c[0]] for c in con}
    lv_h, slot_h, top_h = schedule(gh, list(amap), amap, set(), nacc, uses, hlev)
    vrr = encode([[(k2, gv.nodes[k2]) for k2 in lv] for lv in lv_v], slot_v)
    hrr = encode([[(k2, gh.nodes[k2]) for k2 in lv] for lv in lv_h], slot_h)
    nl = max(len(lv_h) + 1, max(hlev.values()) + 1)
    con_by = [[] for _ in range(nl)]
    for c in con:
        con_by[hlev[c[0]]].append(c)
    con_lstart, flat = [0], []
    for lst in con_by:
        flat += lst
        con_lstart.append(len(flat))
    return dict(L=L, lsh=(la, lb, lc, ld), nslot=max(top_h, top_v), vrr=vrr, hrr=hrr, acc_slot=acc_slot,
                tgt_slot=tgt_slot, tgt_w=tw, nacc=nacc, nout=n, fslot=nacc,
                con_lstart=con_lstart, con_slot=[slot_h[c[0]] for c in flat],
                con_g=[c[1] for c in flat], con_G=[c[2] for c in flat], con_c=[c[3] for c in flat])


def pack_phase(ph):
    """Pack one phase for the device: a 64-bit word per node (first term,
    destination slot, term count) and a 32-bit word per term (source slot,
    scalar selector, multiplier + 8).  Multipliers are small integers."""
    ls, dst, t0, src, sel, mult = ph
    nodes, terms = [], []
    for i, d in enumerate(dst):
        cnt = t0[i + 1] - t0[i]
        assert 0 <= d < 1 << 16 and 0 <= cnt < 1 << 8 and 0 <= t0[i] < 1 << 32
        nodes.append(t0[i] | (d << 32) | (cnt << 48))
    for x, se, m in zip(src, sel, mult):
        assert m == int(m) and -8 <= m < 248 and 0 <= x < 1 << 16 and 0 <= se < 1 << 8
        terms.append(x | (se << 16) | ((int(m) + 8) << 24))
    return list(ls), nodes, terms


def unpack_phase(ls, nodes, terms):
    """Inverse of pack_phase (the decoding the kernels do)."""
    dst = [(w >> 32) & 0xFFFF for w in nodes]
    t0 = [w & 0xFFFFFFFF for w in nodes]
    t0.append(t0[-1] + ((nodes[-1] >> 48) & 0xFF) if nodes else 0)
    src = [u & 0xFFFF for u in terms]
    sel = [(u >> 16) & 0xFF for u in terms]
    mult = [float(((u >> 24) & 0xFF) - 8) for u in terms]
    return list(ls), dst, t0, src, sel, mult


def pack_con(prog):
    """Gradient contraction entries as 64-bit words (slot, G index, gradient
    component, coefficient index) plus the table of distinct coefficients."""
    ctab = sorted(set(prog["con_c"]))
    assert len(ctab) < 256
    words = []
    for sl, gk, G, c in zip(prog["con_slot"], prog["con_g"], prog["con_G"], prog["con_c"]):
        assert 0 <= sl < 1 << 16 and 0 <= G < 1 << 16 and 0 <= gk < 9
        words.append(sl | (G << 16) | (gk << 32) | (ctab.index(c) << 40))
    return words, ctab


def unpack_con(words, ctab):
    return dict(con_slot=[w & 0xFFFF for w in words], con_G=[(w >> 16) & 0xFFFF for w in words],
                con_g=[(w >> 32) & 0xFF for w in words], con_c=[ctab[(w >> 40) & 0xFF] for w in words])


def packed(prog):
    """The program with every table replaced by its decoded packed form."""
    q = dict(prog)
    for ph in ("vrr", "hrr"):
        q[ph] = unpack_phase(*pack_phase(prog[ph]))
    if "con_c" in prog:
        q.update(unpack_con(*pack_con(prog)))
    return q


def lds_doubles(prog, grad):
    """LDS of the cooperative kernels, in doubles (slots, scalars, and the
    density factors (gradient) or the digestion blocks (Fock))."""
    la, lb, lc, ld = prog["lsh"]
    na, nb, nc, nd = (ncart(x) for x in (la, lb, lc, ld))
    extra = na * nb * nc * nd + 16 + 9 * 8 if grad else (na * nb + nc * nd + (na + nb) * (nc + nd))
    return prog["nslot"] + NSEL + extra


def threads_per_block(prog, grad, lds_per_cu=160 * 1024):
    """Threads that share one quartet: enough for about eight wavefronts per
    CU once LDS limits the resident blocks, at most the program's typical
    level width (rounded to wavefronts) and 512."""
    per_cu = max(1, lds_per_cu // (8 * lds_doubles(prog, grad)))
    nt = 64 * -(-8 // per_cu)
    widths = []
    for ph in ("vrr", "hrr"):
        ls = prog[ph][0]
        widths += [ls[i + 1] - ls[i] for i in range(len(ls) - 1)]
    widths.sort()
    med = widths[len(widths) // 2] if widths else 64
    return max(64, min(nt, 512, (med // 64) * 64))


def grad_quartets_per_block(prog, budget=56 * 1024):
    """Quartets per block of the cooperative gradient: the largest power of
    two up to 8 whose LDS stays within `budget` bytes (table loads and the
    per-primitive set-up are shared by the block's quartets)."""
    per = 8 * lds_doubles(prog, True)
    qb = 1
    while qb < 8 and 2 * qb * per <= budget:
        qb *= 2
    return qb


def grad_block_threads(prog):
    """Threads of a cooperative gradient block: the per-quartet count times
    the quartets per block, at most 256 (never fewer than one quartet's)."""
    nt = threads_per_block(prog, True)
    return max(nt, min(256, nt * grad_quartets_per_block(prog)))


def emit_tables(name, prog, grad=False):
    """C++ constant tables of one program (namespace-scope __device__)."""
    def arr(t, nm, v):
        if t == "double":
            body = ", ".join(repr(float(x)) for x in v)
        elif t == "unsigned long long":
            body = ", ".join(f"{int(x)}ull" for x in v)
        else:
            body = ", ".join(str(int(x)) for x in v)
        return f"__device__ const {t} {name}_{nm}[{max(len(v), 1)}] = {{{body or '0'}}};"
    out = [f"// cooperative tables: {prog['nslot']} LDS slots, L = {prog['L']}"]
    # the kernels rely on these: accumulator k in slot k, at most five terms
    # per VRR node and two per HRR node (coop_kernel.h, kVrrTerms / kHrrTerms)
    assert list(prog["acc_slot"]) == list(range(prog["nacc"]))
    for ph, mx in (("vrr", 5), ("hrr", 2)):
        t0 = prog[ph][2]
        assert all(t0[i + 1] - t0[i] <= mx for i in range(len(t0) - 1)), (ph, prog["lsh"])
    for ph in ("vrr", "hrr"):
        ls, nodes, terms = pack_phase(prog[ph])
        out += [arr("int", f"{ph}_lstart", ls), arr("unsigned long long", f"{ph}_node", nodes),
                arr("unsigned int", f"{ph}_term", terms)]
    out += [arr("unsigned short", "acc_slot", prog["acc_slot"]),
            arr("unsigned short", "tgt_slot", prog["tgt_slot"]),
            arr("unsigned char", "tgt_w", prog["tgt_w"])]
    if not grad:
        out += [arr("unsigned short", "out_slot", prog["out_slot"]),
                arr("double", "norm", prog["norms"])]
    else:
        words, ctab = pack_con(prog)
        out += [arr("int", "con_lstart", prog["con_lstart"]),
                arr("unsigned long long", "con_word", words),
                arr("double", "con_ctab", ctab)]
    return "\n".join(out)


def interpret(prog, F_per_prim, scalars_per_prim, hrr_scalars, grad_G=None):
    """Reference interpreter of a program (for CPU checks): F_per_prim and
    scalars_per_prim are lists over primitive quartets."""
    slots = [0.0] * prog["nslot"]
    for k in prog["acc_slot"]:
        slots[k] = 0.0

    g = [0.0] * 9

    def contract(lv):
        if grad_G is None:
            return
        cs = prog["con_lstart"]
        for c in range(cs[lv], cs[lv + 1]):
            g[prog["con_g"][c]] += prog["con_c"][c] * grad_G[prog["con_G"][c]] * slots[prog["con_slot"][c]]

    def run(ph, sc, with_con=False):
        ls, dst, t0, src, sel, mult = prog[ph]
        nlev = len(ls) - 1
        ncon = len(prog["con_lstart"]) - 1 if with_con else 0
        for lv in range(max(nlev + 1, ncon)):
            if 1 <= lv <= nlev:
                new = []
                for nd in range(ls[lv - 1], ls[lv]):
                    v = 0.0
                    for t in range(t0[nd], t0[nd + 1]):
                        v += mult[t] * sc[sel[t]] * slots[src[t]]
                    new.append((dst[nd], v))
                for d, v in new:
                    slots[d] = v
            if lv < ncon:
                contract(lv)

    for F, sc in zip(F_per_prim, scalars_per_prim):
        for m, f in enumerate(F):
            slots[prog["fslot"] + m] = f
        run("vrr", sc)
        for a, t, w in zip(prog["acc_slot"], prog["tgt_slot"], prog["tgt_w"]):
            slots[a] += sc[w] * slots[t]
    run("hrr", hrr_scalars, with_con=grad_G is not None)
    if grad_G is None:
        return [slots[s] * n for s, n in zip(prog["out_slot"], prog["norms"])]
    return g
