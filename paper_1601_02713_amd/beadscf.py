"""Thin ctypes binding of libbeadscf.so (include/beadscf.h).

Argument marshalling only: every step of the energy/force path runs in the
library's HIP kernels.  Importing this module without the built library raises
ImportError; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbeadscf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1601_02713_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

BSCF_FP64, BSCF_MIXED = 0, 1
GUESS_CORE, GUESS_PREVIOUS, GUESS_LEARNED, GUESS_USER, GUESS_EXTRAPOLATED = 0, 1, 2, 3, 4
DENSITY_SP2, DENSITY_EIG = 0, 1
STATUS_MAX_ITER, STATUS_NAN, STATUS_FALLBACK = 1, 2, 4
XC_NONE, XC_B3LYP = 0, 1


class ScfOpts(ctypes.Structure):
    _fields_ = [("e_tol", ctypes.c_double), ("comm_tol", ctypes.c_double),
                ("schwarz_tol", ctypes.c_double), ("fp32_split_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("diis_size", ctypes.c_int),
                ("precision", ctypes.c_int), ("guess", ctypes.c_int),
                ("deterministic", ctypes.c_int), ("density", ctypes.c_int),
                ("incremental", ctypes.c_int), ("graph", ctypes.c_int)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_SIGS = {
    "bscf_default_opts": [ctypes.POINTER(ScfOpts)],
    "bscf_create": [_i, _vp, ctypes.POINTER(_vp)],
    "bscf_destroy": [_vp],
    "bscf_load_basis": [_vp, ctypes.c_char_p],
    "bscf_set_instances": [_vp, _i, _vp, _vp, _vp],
    "bscf_set_geometries": [_vp, _vp],
    "bscf_build_fock": [_vp, _vp, _vp, _vp, _d, _i, _i],
    "bscf_build_jk": [_vp, _vp, _vp, _vp, _d, _i, _i],
    "bscf_run_scf": [_vp, ctypes.POINTER(ScfOpts), _vp, _vp, _vp],
    "bscf_forces": [_vp, _vp],
    "bscf_forces_at": [_vp, _vp, _vp, _vp, _d, _i],
    "bscf_get_density": [_vp, _i, _vp, _i],
    "bscf_set_density": [_vp, _vp, _i],
    "bscf_get_one_electron": [_vp, _i, _vp, _vp],
    "bscf_eri_tensor": [_vp, _i, _vp],
    "bscf_schwarz": [_vp, _i, _vp, _i],
    "bscf_instance_info": [_vp, _i, _vp, _vp, _vp],
    "bscf_work_counts": [_vp, _vp, _vp, _vp],
    "bscf_get_stats": [_vp, ctypes.c_char_p, _i],
    "bscf_set_profiling": [_vp, _i],
    "bscf_set_deterministic": [_vp, _i],
    "bscf_reset_stats": [_vp],
    "bscf_boys": [_vp, _i, _i, _vp, _vp, _i],
    "bscf_guess_train": [_vp, _i, _vp],
    "bscf_checkpoint_save": [_vp, ctypes.c_char_p],
    "bscf_checkpoint_load": [_vp, ctypes.c_char_p],
    "bscf_guess_save": [_vp, ctypes.c_char_p],
    "bscf_guess_load": [_vp, ctypes.c_char_p],
    "bscf_guess_configure": [_vp, _i, _i, ctypes.c_uint],
    "bscf_guess_param_count": [_vp, _vp, _vp, _vp],
    "bscf_guess_set_params": [_vp, _vp, ctypes.c_long],
    "bscf_guess_get_params": [_vp, _vp, ctypes.c_long],
    "bscf_guess_eval": [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp],
    "bscf_guess_fit": [_vp, _i, _vp, _vp, _vp, _i, ctypes.c_float, _vp],
    "bscf_guess_eval_noalloc": [_vp, _i, _vp, _vp],
    "bscf_set_xc": [_vp, _i],
    "bscf_xc_matrix": [_vp, _vp, _vp, _vp, _i],
    "bscf_xc_grid_size": [_vp, _i, _vp],
    "bscf_xc_functional": [_vp, _i, _vp, _vp, _vp, _vp, _vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.bscf_last_error.restype = ctypes.c_char_p
_lib.bscf_last_error.argtypes = []
_lib.bscf_boys_table_entry.restype = ctypes.c_double
_lib.bscf_boys_table_entry.argtypes = [_i, _i]


class PimdOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("temperature", ctypes.c_double),
                ("thermostat", ctypes.c_int), ("tau_centroid", ctypes.c_double),
                ("friction_scale", ctypes.c_double), ("seed", ctypes.c_ulonglong)]


_SIGS.update({
    "bscf_pimd_default_opts": [ctypes.POINTER(PimdOpts)],
    "bscf_pimd_init": [_vp, ctypes.POINTER(PimdOpts), _vp, _vp],
    "bscf_pimd_step": [_vp, ctypes.POINTER(ScfOpts), _vp, _vp, _vp, _vp],
    "bscf_pimd_begin": [_vp, _vp],
    "bscf_pimd_end": [_vp, _vp],
    "bscf_pimd_state": [_vp, _vp, _vp, _vp],
})
for _name in ("bscf_pimd_default_opts", "bscf_pimd_init", "bscf_pimd_step", "bscf_pimd_begin",
              "bscf_pimd_end", "bscf_pimd_state"):
    _f = getattr(_lib, _name)
    _f.argtypes = _SIGS[_name]
    _f.restype = ctypes.c_int


class StringOpts(ctypes.Structure):
    _fields_ = [("step", ctypes.c_double), ("fix_ends", ctypes.c_int)]


_SIGS.update({
    "bscf_string_default_opts": [ctypes.POINTER(StringOpts)],
    "bscf_string_init": [_vp, ctypes.POINTER(StringOpts)],
    "bscf_string_step": [_vp, ctypes.POINTER(ScfOpts), _vp, _vp, _vp, _vp],
    "bscf_string_evolve": [_vp, _vp],
    "bscf_string_state": [_vp, _vp, _vp],
})
for _name in ("bscf_string_default_opts", "bscf_string_init", "bscf_string_step",
              "bscf_string_evolve", "bscf_string_state"):
    _f = getattr(_lib, _name)
    _f.argtypes = _SIGS[_name]
    _f.restype = ctypes.c_int


def string_default_opts(**kw) -> StringOpts:
    o = StringOpts()
    _chk(_lib.bscf_string_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def pimd_default_opts(**kw) -> PimdOpts:
    o = PimdOpts()
    _chk(_lib.bscf_pimd_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class BscfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"beadscf error {code}: {msg}")
        self.code = code


def _chk(rc):
    if rc != 0:
        raise BscfError(rc, _lib.bscf_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(_vp)


def default_opts(**kw) -> ScfOpts:
    o = ScfOpts()
    _chk(_lib.bscf_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def boys_table_entry(m: int, k: int) -> float:
    return _lib.bscf_boys_table_entry(m, k)


def exported_symbols():
    return list(_SIGS) + ["bscf_last_error", "bscf_boys_table_entry"]


class Engine:
    """One context on one HIP device (optionally on a caller's stream)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        h = _vp()
        _chk(_lib.bscf_create(device, _vp(stream) if stream else None, ctypes.byref(h)))
        self._h = h
        self.n_inst = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.bscf_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---- setup
    def load_basis(self, basis):
        text = basis if isinstance(basis, str) else json.dumps(basis)
        _chk(_lib.bscf_load_basis(self._h, text.encode()))

    def set_instances(self, Zs, charges=None):
        Zs = [np.asarray(z, np.int32) for z in Zs]
        na = np.array([len(z) for z in Zs], np.int32)
        zc = np.ascontiguousarray(np.concatenate(Zs).astype(np.int32))
        ch = None if charges is None else np.ascontiguousarray(np.asarray(charges, np.int32))
        _chk(_lib.bscf_set_instances(self._h, len(Zs), _ptr(na), _ptr(zc),
                                     _ptr(ch) if ch is not None else None))
        self.n_inst = len(Zs)
        self.natoms = na
        self.nbf = []
        for i in range(self.n_inst):
            nb = ctypes.c_int()
            _chk(_lib.bscf_instance_info(self._h, i, ctypes.byref(nb), None, None))
            self.nbf.append(nb.value)

    def set_geometries(self, xyzs):
        x = np.ascontiguousarray(np.concatenate([np.asarray(v, float).reshape(-1, 3) for v in xyzs]))
        _chk(_lib.bscf_set_geometries(self._h, _ptr(x)))

    def _cat(self, mats):
        mats = [np.asarray(m, float) for m in mats]
        if [m.shape for m in mats] != [(n, n) for n in self.nbf]:
            raise ValueError(f"expected matrices of shapes {[(n, n) for n in self.nbf]}")
        return np.ascontiguousarray(np.concatenate([m.ravel() for m in mats]))

    def _split(self, flat):
        out, o = [], 0
        for n in self.nbf:
            out.append(flat[o:o + n * n].reshape(n, n).copy())
            o += n * n
        return out

    # ---- compute
    def build_fock(self, Ps, schwarz_tol=1e-12, precision=BSCF_FP64):
        P = self._cat(Ps)
        F = np.empty_like(P)
        E = np.empty(self.n_inst)
        _chk(_lib.bscf_build_fock(self._h, _ptr(P), _ptr(F), _ptr(E), schwarz_tol, precision, 0))
        return self._split(F), E

    def build_jk(self, Ps, schwarz_tol=1e-12, precision=BSCF_FP64):
        P = self._cat(Ps)
        J, K = np.empty_like(P), np.empty_like(P)
        _chk(_lib.bscf_build_jk(self._h, _ptr(P), _ptr(J), _ptr(K), schwarz_tol, precision, 0))
        return self._split(J), self._split(K)

    def run_scf(self, opts: ScfOpts | None = None, **kw):
        o = opts or default_opts(**kw)
        E = np.empty(self.n_inst)
        it = np.empty(self.n_inst, np.int32)
        st = np.empty(self.n_inst, np.int32)
        _chk(_lib.bscf_run_scf(self._h, ctypes.byref(o), _ptr(E), _ptr(it), _ptr(st)))
        return E, it, st

    def forces(self):
        F = np.empty((int(self.natoms.sum()), 3))
        _chk(_lib.bscf_forces(self._h, _ptr(F)))
        out, o = [], 0
        for n in self.natoms:
            out.append(F[o:o + n].copy())
            o += n
        return out

    def forces_at(self, Ps, Fs, schwarz_tol=1e-12):
        """-dE/dR per instance at caller densities and Fock matrices."""
        P, Fm = self._cat(Ps), self._cat(Fs)
        G = np.empty((int(self.natoms.sum()), 3))
        _chk(_lib.bscf_forces_at(self._h, _ptr(P), _ptr(Fm), _ptr(G), schwarz_tol, 0))
        out, o = [], 0
        for n in self.natoms:
            out.append(G[o:o + n].copy())
            o += n
        return out

    # ---- ring polymer (the batch's instances are its beads)
    def pimd_init(self, masses, p0=None, opts: PimdOpts | None = None, **kw):
        o = opts or pimd_default_opts(**kw)
        m = np.ascontiguousarray(np.asarray(masses, float))
        p = None if p0 is None else np.ascontiguousarray(np.asarray(p0, float))
        if p is not None and p.size != 3 * int(self.natoms.sum()):
            raise ValueError("p0 must hold [P][n_atoms][3] momenta")
        if m.size != int(self.natoms[0]):
            raise ValueError("one mass per atom of a bead")
        _chk(_lib.bscf_pimd_init(self._h, ctypes.byref(o), _ptr(m), _ptr(p) if p is not None else None))

    def pimd_step(self, opts: ScfOpts | None = None, return_forces=False, **kw):
        """One MD step; (E, iterations, status) of the new positions, and
        with return_forces their forces per bead."""
        o = opts or default_opts(**kw)
        E = np.empty(self.n_inst)
        it = np.empty(self.n_inst, np.int32)
        st = np.empty(self.n_inst, np.int32)
        F = np.empty((int(self.natoms.sum()), 3)) if return_forces else None
        _chk(_lib.bscf_pimd_step(self._h, ctypes.byref(o), _ptr(E), _ptr(it), _ptr(st),
                                 _ptr(F) if F is not None else None))
        if not return_forces:
            return E, it, st
        n = int(self.natoms[0])
        return E, it, st, [F[k * n:(k + 1) * n].copy() for k in range(self.n_inst)]

    def _pimd_forces(self, F):
        if F is None:
            return None
        F = np.ascontiguousarray(np.asarray(F, float))
        if F.size != 3 * int(self.natoms.sum()):
            raise ValueError("forces must be [P][n_atoms][3]")
        return F

    def pimd_begin(self, F=None):
        F = self._pimd_forces(F)
        _chk(_lib.bscf_pimd_begin(self._h, _ptr(F) if F is not None else None))

    def pimd_end(self, F=None):
        F = self._pimd_forces(F)
        _chk(_lib.bscf_pimd_end(self._h, _ptr(F) if F is not None else None))

    def pimd_state(self):
        """(x, p [P, N, 3], kinetic, spring, steps)."""
        P, N = self.n_inst, int(self.natoms[0])
        x, p, obs = np.empty((P, N, 3)), np.empty((P, N, 3)), np.empty(3)
        _chk(_lib.bscf_pimd_state(self._h, _ptr(x), _ptr(p), _ptr(obs)))
        return x, p, float(obs[0]), float(obs[1]), int(obs[2])

    # ---- checkpoint / resume between steps
    def checkpoint_save(self, path):
        _chk(_lib.bscf_checkpoint_save(self._h, str(path).encode()))

    def checkpoint_load(self, path):
        _chk(_lib.bscf_checkpoint_load(self._h, str(path).encode()))

    # ---- string method (the batch's instances are its images)
    def string_init(self, opts: StringOpts | None = None, **kw):
        o = opts or string_default_opts(**kw)
        _chk(_lib.bscf_string_init(self._h, ctypes.byref(o)))

    def string_step(self, opts: ScfOpts | None = None, **kw):
        """One iteration; (E, iterations, status, forces) of the images as
        evaluated, before they moved."""
        o = opts or default_opts(**kw)
        E = np.empty(self.n_inst)
        it = np.empty(self.n_inst, np.int32)
        st = np.empty(self.n_inst, np.int32)
        n = int(self.natoms[0])
        F = np.empty((self.n_inst, n, 3))
        _chk(_lib.bscf_string_step(self._h, ctypes.byref(o), _ptr(E), _ptr(it), _ptr(st), _ptr(F)))
        return E, it, st, F

    def string_evolve(self, F):
        F = np.ascontiguousarray(np.asarray(F, float))
        if F.size != 3 * int(self.natoms.sum()):
            raise ValueError("forces must be [n][n_atoms][3]")
        _chk(_lib.bscf_string_evolve(self._h, _ptr(F)))

    def string_state(self):
        """(images [n, N, 3], normalised arc positions [n])."""
        x = np.empty((self.n_inst, int(self.natoms[0]), 3))
        s = np.empty(self.n_inst)
        _chk(_lib.bscf_string_state(self._h, _ptr(x), _ptr(s)))
        return x, s

    def density(self, i):
        n = self.nbf[i]
        P = np.empty((n, n))
        _chk(_lib.bscf_get_density(self._h, i, _ptr(P), 0))
        return P

    def set_density(self, Ps):
        P = self._cat(Ps)
        _chk(_lib.bscf_set_density(self._h, _ptr(P), 0))

    def one_electron(self, i):
        n = self.nbf[i]
        S, H = np.empty((n, n)), np.empty((n, n))
        _chk(_lib.bscf_get_one_electron(self._h, i, _ptr(S), _ptr(H)))
        return S, H

    def eri_tensor(self, i):
        n = self.nbf[i]
        out = np.empty((n, n, n, n))
        _chk(_lib.bscf_eri_tensor(self._h, i, _ptr(out)))
        return out

    def schwarz(self, i):
        ns = ctypes.c_int()
        _chk(_lib.bscf_instance_info(self._h, i, None, ctypes.byref(ns), None))
        Q = np.empty((ns.value, ns.value))
        _chk(_lib.bscf_schwarz(self._h, i, _ptr(Q), ns.value))
        return Q

    def work_counts(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _chk(_lib.bscf_work_counts(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_xc(self, functional=XC_B3LYP):
        """XC_NONE (Hartree-Fock) or XC_B3LYP for later Fock builds and SCFs."""
        _chk(_lib.bscf_set_xc(self._h, int(functional)))

    def xc_matrix(self, Ps):
        """(V_xc per instance, E_xc [n_inst]) of B3LYP at densities Ps."""
        P = self._cat(Ps)
        V = np.empty_like(P)
        E = np.empty(self.n_inst)
        _chk(_lib.bscf_xc_matrix(self._h, _ptr(P), _ptr(V), _ptr(E), 0))
        return self._split(V), E

    def xc_grid_size(self, i):
        n = ctypes.c_longlong()
        _chk(_lib.bscf_xc_grid_size(self._h, i, ctypes.byref(n)))
        return n.value

    def xc_functional(self, rho, sigma):
        """(e, v_rho, v_sigma) of the closed-shell B3LYP energy density."""
        rho = np.ascontiguousarray(np.asarray(rho, float))
        sigma = np.ascontiguousarray(np.asarray(sigma, float))
        if rho.shape != sigma.shape or rho.ndim != 1:
            raise ValueError("rho and sigma must be 1-D arrays of one length")
        e, vr, vs = np.empty_like(rho), np.empty_like(rho), np.empty_like(rho)
        _chk(_lib.bscf_xc_functional(self._h, len(rho), _ptr(rho), _ptr(sigma), _ptr(e), _ptr(vr),
                                     _ptr(vs)))
        return e, vr, vs

    def set_deterministic(self, on=True):
        _chk(_lib.bscf_set_deterministic(self._h, 1 if on else 0))

    def set_profiling(self, on=True):
        _chk(_lib.bscf_set_profiling(self._h, 1 if on else 0))

    def reset_stats(self):
        _chk(_lib.bscf_reset_stats(self._h))

    def stats(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _chk(_lib.bscf_get_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def boys(self, m_max, T, precision=0):
        T = np.ascontiguousarray(np.asarray(T, float))
        out = np.empty((len(T), m_max + 1))
        _chk(_lib.bscf_boys(self._h, m_max, len(T), _ptr(T), _ptr(out), precision))
        return out

    def guess_train(self, steps):
        l = ctypes.c_float()
        _chk(_lib.bscf_guess_train(self._h, steps, ctypes.byref(l)))
        return l.value

    def guess_save(self, path):
        _chk(_lib.bscf_guess_save(self._h, path.encode()))

    def guess_load(self, path):
        _chk(_lib.bscf_guess_load(self._h, path.encode()))

    def guess_configure(self, din, dout, seed=2000):
        _chk(_lib.bscf_guess_configure(self._h, din, dout, seed))

    def guess_dims(self):
        di, do, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
        _chk(_lib.bscf_guess_param_count(self._h, ctypes.byref(di), ctypes.byref(do), ctypes.byref(n)))
        return di.value, do.value, n.value

    def guess_params(self):
        n = self.guess_dims()[2]
        p = np.empty(n, np.float32)
        _chk(_lib.bscf_guess_get_params(self._h, _ptr(p), n))
        return p

    def guess_set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, np.float32))
        _chk(_lib.bscf_guess_set_params(self._h, _ptr(p), p.size))

    def guess_eval_noalloc(self, rows, x_dev_ptr, y_dev_ptr):
        """Allocation-free evaluation on device buffers (addresses as ints),
        enqueued on the context's stream without synchronising."""
        _chk(_lib.bscf_guess_eval_noalloc(self._h, rows, _vp(x_dev_ptr), _vp(y_dev_ptr)))

    def guess_eval(self, X, T=None, mask=None):
        """(Y, gradient, loss) of the network on host rows; gradient and loss
        are None without targets."""
        X = np.ascontiguousarray(np.asarray(X, np.float32))
        _, dout, n = self.guess_dims()
        Y = np.empty((X.shape[0], dout), np.float32)
        if T is None:
            _chk(_lib.bscf_guess_eval(self._h, X.shape[0], _ptr(X), None, None, _ptr(Y), None, None))
            return Y, None, None
        T = np.ascontiguousarray(np.asarray(T, np.float32))
        M = np.ascontiguousarray(np.asarray(mask, np.float32))
        g = np.empty(n, np.float32)
        l = ctypes.c_float()
        _chk(_lib.bscf_guess_eval(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(M), _ptr(Y), _ptr(g),
                                  ctypes.byref(l)))
        return Y, g, l.value

    def guess_fit(self, X, T, mask, steps, lr=1e-3):
        X = np.ascontiguousarray(np.asarray(X, np.float32))
        T = np.ascontiguousarray(np.asarray(T, np.float32))
        M = np.ascontiguousarray(np.asarray(mask, np.float32))
        l = ctypes.c_float()
        _chk(_lib.bscf_guess_fit(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(M), steps, lr,
                                 ctypes.byref(l)))
        return l.value
