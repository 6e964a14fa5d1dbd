"""Oracle multigrid (plain FP64 C, see ``mg_oracle.c``) and its ctypes wrapper.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path.
"""
import ctypes
import sys
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_mg.so")
SRC = os.path.join(HERE, "mg_oracle.c")

PHI, RHS, OLD, RES = 0, 1, 2, 3
IDX_ORDER, IDX_LEVEL, IDX_IJK, IDX_TREE, IDX_PARENT, IDX_CHILD, IDX_NBR, IDX_CFQ = range(8)
OP_SMOOTH, OP_FAS_DOWN, OP_PROLONG, OP_COARSE, OP_RESTRICT_ALL, OP_VCYCLE, OP_RESIDUAL = range(1, 8)
CODES = {0: "OK", -1: "EINVAL", -2: "ENESTING", -3: "ENOMEM", -5: "ENOCONV", -6: "ESTATE",
         -7: "ETOPO"}
_WIDTH = {IDX_ORDER: 1, IDX_LEVEL: 1, IDX_IJK: 3, IDX_TREE: 1, IDX_PARENT: 1, IDX_CHILD: 8,
          IDX_NBR: 6, IDX_CFQ: 6}


def build(force=True):
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O3", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
           "-shared", "-fPIC", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oracle_create.argtypes = [ctypes.POINTER(P), I64, P, P, P, P, D, P, P]
        L.oracle_destroy.argtypes = [P]
        L.oracle_destroy.restype = None
        L.oracle_info.argtypes = [P, P]
        L.oracle_index.argtypes = [P, I32, P]
        L.oracle_set_field.argtypes = [P, I32, P]
        L.oracle_get_field.argtypes = [P, I32, P]
        L.oracle_set_bcval.argtypes = [P, P]
        L.oracle_fmg_solve.argtypes = [P, D, I32, I32, I32, P]
        L.oracle_vcycles.argtypes = [P, I32, D, I32, I32, P]
        L.oracle_residual.argtypes = [P, P]
        L.oracle_step.argtypes = [P, I32, I32, I32]
        L.oracle_apply.argtypes = [P, P, P, I32]
        L.oracle_set_threads.argtypes = [I32]
        L.oracle_tree_rel.argtypes = [P, P]
        L.oracle_efield.argtypes = [P, P, P]
        L.oracle_transfer.argtypes = [P, P]
        L.oracle_koren_psi.argtypes = [D]
        L.oracle_koren_psi.restype = D
        L.oracle_fluid_coeffs.argtypes = [P, I32, D, D, P]
        L.oracle_fluid_coeffs.restype = None
        L.oracle_fluid_stage.argtypes = [P, P, P, P, P, P, P, P, I32, D, D, D, D, P, P, P]
        L.oracle_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODES.get(code, code)}: {msg}")
        self.code = code
        self.name = CODES.get(code, str(code))


def _check(rc):
    if rc != 0:
        raise OracleError(rc, lib().oracle_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n):
    return lib().oracle_set_threads(int(n))


class OracleTree:
    """One octree (or forest) with its fields, in the oracle's canonical order
    (level, tree, Morton index)."""

    def __init__(self, level, ijk, tree=None, lo=(0.0, 0.0, 0.0), length=1.0,
                 bc_type=(0,) * 6, bc_val=(0.0,) * 6):
        self._keep = [np.ascontiguousarray(level, dtype=np.int32),
                      np.ascontiguousarray(np.asarray(ijk).reshape(-1, 3), dtype=np.int32),
                      None if tree is None else np.ascontiguousarray(tree, dtype=np.int32),
                      np.ascontiguousarray(lo, dtype=np.float64),
                      np.ascontiguousarray(bc_type, dtype=np.int32),
                      np.ascontiguousarray(bc_val, dtype=np.float64)]
        lv, ij, tr, lo_, bt, bv = self._keep
        h = ctypes.c_void_p()
        _check(lib().oracle_create(ctypes.byref(h), len(lv), _ptr(lv), _ptr(ij),
                                   None if tr is None else _ptr(tr), _ptr(lo_), float(length),
                                   _ptr(bt), _ptr(bv)))
        self.h = h
        info = np.zeros(24, dtype=np.int64)
        _check(lib().oracle_info(self.h, _ptr(info)))
        self.n, self.nlev, self.ntree, self.n_leaf_boxes = (int(v) for v in info[:4])
        self.level_start = info[4:4 + self.nlev + 1].copy()  # boxes of level l: [ls[l-1], ls[l])
        self.length = float(length)

    @classmethod
    def from_workload(cls, w):
        b = w.boxes
        return cls(b.level, b.ijk, b.tree, w.lo, w.length, w.bc_type, w.bc_val)

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "h", None)
        if not h:
            return
        self.h = None
        if _finalizing():
            return  # process exit releases the memory; module globals may already be gone
        lib().oracle_destroy(h)

    def index(self, what):
        out = np.zeros((self.n, _WIDTH[what]), dtype=np.int32)
        _check(lib().oracle_index(self.h, what, _ptr(out)))
        return out if _WIDTH[what] > 1 else out[:, 0]

    def set_field(self, which, nat):
        a = np.ascontiguousarray(nat, dtype=np.float64).reshape(self.n, 8, 8, 8)
        _check(lib().oracle_set_field(self.h, which, _ptr(a)))

    def get_field(self, which):
        a = np.zeros((self.n, 8, 8, 8))
        _check(lib().oracle_get_field(self.h, which, _ptr(a)))
        return a

    def set_bcval(self, vals):
        if vals is None:
            _check(lib().oracle_set_bcval(self.h, None))
            return
        a = np.ascontiguousarray(vals, dtype=np.float64).reshape(self.n, 6, 64)
        _check(lib().oracle_set_bcval(self.h, _ptr(a)))

    def set_rhs_from(self, w):
        """Evaluate the workload's right-hand side at this tree's boxes."""
        lv = self.index(IDX_LEVEL)
        ij = self.index(IDX_IJK)
        self.set_field(RHS, w.rhs(lv, ij, self.index(IDX_TREE)))

    def fmg_solve(self, tol=1e-8, max_cycles=50, n_down=2, n_up=2):
        st = np.zeros(69)
        rc = lib().oracle_fmg_solve(self.h, tol, max_cycles, n_down, n_up, _ptr(st))
        _check(rc)
        return _stats(st)

    def vcycles(self, n, tol=1e-8, n_down=2, n_up=2):
        st = np.zeros(69)
        _check(lib().oracle_vcycles(self.h, n, tol, n_down, n_up, _ptr(st)))
        return _stats(st)

    def residual(self):
        out = np.zeros(4)
        _check(lib().oracle_residual(self.h, _ptr(out)))
        return dict(rel=out[0], l2=out[1], linf=out[2], beff=out[3])

    def tree_rel(self):
        out = np.zeros(self.ntree)
        _check(lib().oracle_tree_rel(self.h, _ptr(out)))
        return out

    def step(self, op, level=0, arg=0):
        _check(lib().oracle_step(self.h, op, level, arg))

    def apply(self, x, homog=True):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        _check(lib().oracle_apply(self.h, _ptr(x), _ptr(y), int(homog)))
        return y

    def transfer_from(self, other):
        """phi of this tree from another over the same domain (regrid step):
        common boxes copied, new boxes interpolated from their parents."""
        _check(lib().oracle_transfer(other.h, self.h))

    def efield(self):
        """Electric field of the current phi (covered cells reset to the mean
        of their children first): face components [n][3][9][8][8] (axis,
        face index, second then first tangential axis) and the cell-centre
        strength [n][8][8][8] (natural order)."""
        face = np.zeros((self.n, 3, 9, 8, 8))
        norm = np.zeros((self.n, 8, 8, 8))
        _check(lib().oracle_efield(self.h, _ptr(face), _ptr(norm)))
        return face, norm

    def fluid_stage(self, ne, ni, n0e, n0i, e_face, e_norm, table, emax, dt, wa=0.0, wb=1.0):
        """One explicit stage of the fluid model (paper sections 2.2-2.4) on the
        leaf cells: out = wa * n0 + wb * (n + dt * rate(n)); densities
        [n][8][8][8] in SI units, table [ntab][3] = (mu, D, alpha) at
        E = k * emax / (ntab - 1).  Also sets this tree's right-hand side on
        the leaf cells to -e (n_i - n_e) / eps0 of the output.  Returns
        (out_e, out_i, dt limit); non-leaf boxes of the outputs keep the
        input values."""
        arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (ne, ni, n0e, n0i, e_face, e_norm)]
        tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 3)
        oe, oi = arr[0].copy(), arr[1].copy()
        lim = np.zeros(1)
        _check(lib().oracle_fluid_stage(self.h, *[_ptr(x) for x in arr], _ptr(tab), len(tab),
                                        float(emax), float(dt), float(wa), float(wb), _ptr(oe),
                                        _ptr(oi), _ptr(lim)))
        return oe, oi, float(lim[0])

    def fluid_step(self, ne, ni, dt, table, emax, n_vcycles=2, safety=0.9):
        """One time step of the paper's explicit trapezoidal scheme (section
        2.4): keep n, a forward Euler stage over dt, a new field (n_vcycles
        warm-started V-cycles), a second Euler stage, the average of its
        result with the kept densities, a new field.  phi must be the
        potential of (ne, ni) on entry.  Returns (ne, ni, next dt = safety x
        the limit evaluated in the second stage)."""
        ef, en = self.efield()
        n1e, n1i, _ = self.fluid_stage(ne, ni, ne, ni, ef, en, table, emax, dt, 0.0, 1.0)
        self.vcycles(n_vcycles, tol=0.0)
        ef, en = self.efield()
        oe, oi, lim = self.fluid_stage(n1e, n1i, ne, ni, ef, en, table, emax, dt, 0.5, 0.5)
        self.vcycles(n_vcycles, tol=0.0)
        return oe, oi, safety * lim

    def leaf_mask(self):
        return self.index(IDX_CHILD)[:, 0] < 0

    def cell_centres(self, lo=(0.0, 0.0, 0.0)):
        """x, y, z of every cell, [n][8][8][8], for this tree's canonical order."""
        lv = self.index(IDX_LEVEL).astype(np.float64)
        ij = self.index(IDX_IJK).astype(np.float64)
        h = self.length / (8.0 * 2.0 ** (lv - 1))
        loc = np.arange(8) + 0.5
        x = lo[0] + (8 * ij[:, 0])[:, None, None, None] * h[:, None, None, None] \
            + loc[None, None, None, :] * h[:, None, None, None]
        y = lo[1] + (8 * ij[:, 1])[:, None, None, None] * h[:, None, None, None] \
            + loc[None, None, :, None] * h[:, None, None, None]
        z = lo[2] + (8 * ij[:, 2])[:, None, None, None] * h[:, None, None, None] \
            + loc[None, :, None, None] * h[:, None, None, None]
        shape = (self.n, 8, 8, 8)
        return (np.broadcast_to(x, shape), np.broadcast_to(y, shape), np.broadcast_to(z, shape),
                h)


def _stats(st):
    n = int(st[4])
    return dict(rel=st[0], l2=st[1], linf=st[2], beff=st[3], n_vcycles=n,
                hist=st[5:5 + n + 1].copy())
