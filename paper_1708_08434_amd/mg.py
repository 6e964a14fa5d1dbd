"""ctypes binding of libmg.so (declared in include/mg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies the device workspace and the stream.  There is no
fallback: if libmg.so is missing or fails to load, this module raises.
"""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

MG_OK, MG_EINVAL, MG_ENESTING, MG_ENOMEM, MG_EHIP, MG_ENOCONV, MG_ESTATE, MG_ETOPO = \
    0, -1, -2, -3, -4, -5, -6, -7
CODES = {0: "OK", -1: "EINVAL", -2: "ENESTING", -3: "ENOMEM", -4: "EHIP", -5: "ENOCONV",
         -6: "ESTATE", -7: "ETOPO"}
MG_DIRICHLET, MG_NEUMANN = 0, 1
MG_IDX_ORDER, MG_IDX_LEVEL, MG_IDX_IJK, MG_IDX_TREE, MG_IDX_PARENT, MG_IDX_CHILD, MG_IDX_NBR, \
    MG_IDX_CFQ = range(8)
MG_FIELD_PHI, MG_FIELD_RHS, MG_FIELD_OLD, MG_FIELD_BCVAL, MG_FIELD_E32, MG_FIELD_R32, \
    MG_FIELD_OLD32 = range(7)
MG_FP64, MG_MIXED, MG_LEARNED = 0, 1, 2
MG_DTYPE_F64, MG_DTYPE_F32 = 0, 1
MG_OP_SMOOTH, MG_OP_FAS_DOWN, MG_OP_PROLONG, MG_OP_COARSE, MG_OP_RESTRICT_ALL, MG_OP_VCYCLE = \
    range(1, 7)
MG_OP_F32 = 0x100
MG_FUSE_PROLONG = 1
MG_FUSE_BEFF = 2
MG_FUSE_RESTRICT = 4
MG_FUSE_IR = 8
MG_FUSE_ALL = 15
MG_GSRB_VARIANTS = 14  # launch variants: 6, 7 fused sweeps, 8, 9 octets, 10-13 persistent
MG_GSRB_FUSED = (6, 7)
MG_GSRB_OCTET = (8, 9)
MG_GSRB_PERSISTENT = (10, 11, 12, 13)
_WIDTH = {MG_IDX_ORDER: 1, MG_IDX_LEVEL: 1, MG_IDX_IJK: 3, MG_IDX_TREE: 1, MG_IDX_PARENT: 1,
          MG_IDX_CHILD: 8, MG_IDX_NBR: 6, MG_IDX_CFQ: 6}

EXPORTS = ["mg_tree_create", "mg_tree_destroy", "mg_tree_info", "mg_tree_bind", "mg_tree_index",
           "mg_field_set", "mg_field_get", "mg_default_opts", "mg_fmg_solve", "mg_vcycle",
           "mg_residual", "mg_tree_residuals", "mg_step", "mg_timing_enable", "mg_timing_read",
           "mg_autotune", "mg_set_schedule", "mg_stream_copy", "mg_efield", "mg_refine_scores",
           "mg_refine_near", "mg_regrid_plan", "mg_regrid_plan_near", "mg_transfer",
           "mg_fluid_workspace_bytes", "mg_fluid_bind", "mg_fluid_stage", "mg_fluid_step", "mg_set_fusion",
           "mg_field", "mg_last_error"]


class mg_domain(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("len", ctypes.c_double),
                ("bc_type", ctypes.c_int32 * 6), ("bc_val", ctypes.c_double * 6),
                ("per_cell_bc", ctypes.c_int32)]


class mg_tree_info_t(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("n_trees", ctypes.c_int32), ("n_leaf_boxes", ctypes.c_int64),
                ("n_leaf_cells", ctypes.c_int64), ("n_cf_faces", ctypes.c_int64),
                ("level_start", ctypes.c_int64 * 17), ("workspace_bytes", ctypes.c_int64)]


class mg_solve_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_down", ctypes.c_int32),
                ("n_up", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("rel_tol", ctypes.c_double), ("graphs", ctypes.c_int32),
                ("final_check_only", ctypes.c_int32), ("learned_placement", ctypes.c_int32)]


_WS_ROUND = 64 << 20  # workspace allocations are rounded up to this


class mg_solve_stats(ctypes.Structure):
    _fields_ = [("n_vcycles", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("l2", ctypes.c_double), ("linf", ctypes.c_double),
                ("beff_l2", ctypes.c_double), ("rel_hist", ctypes.c_double * 64),
                ("t_ms", ctypes.c_double), ("nn_accepted", ctypes.c_int32),
                ("nn_fell_back", ctypes.c_int32), ("launches_fmg", ctypes.c_int32),
                ("launches_cycle", ctypes.c_int32)]

    def as_dict(self):
        n = self.n_vcycles
        return dict(n_vcycles=n, status=self.status, rel=self.rel_res, l2=self.l2,
                    linf=self.linf, beff=self.beff_l2, hist=np.array(self.rel_hist[:n + 1]),
                    t_ms=self.t_ms, nn_accepted=self.nn_accepted, nn_fell_back=self.nn_fell_back,
                    launches_fmg=self.launches_fmg, launches_cycle=self.launches_cycle)


class mg_kernel_timing_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("level_launches", ctypes.c_int64 * 16),
                ("level_ms", ctypes.c_double * 16), ("level_bytes", ctypes.c_double * 16)]


_lib = None


def lib():
    """Load libmg.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1708_08434_amd/build.py")
        # torch loads its own copy of the HIP runtime (same soname); loading
        # it first makes libmg bind to that copy, so one process holds a
        # single HIP runtime and shares devices and streams with torch.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.mg_tree_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(mg_domain), I64, P, P, P]
        L.mg_tree_destroy.argtypes = [P]
        L.mg_tree_info.argtypes = [P, ctypes.POINTER(mg_tree_info_t)]
        L.mg_tree_bind.argtypes = [P, P, I64, P]
        L.mg_tree_index.argtypes = [P, I32, P]
        L.mg_field_set.argtypes = [P, I32, P]
        L.mg_field_get.argtypes = [P, I32, P]
        L.mg_field.argtypes = [P, I32, I32, ctypes.POINTER(P), ctypes.POINTER(I64), P]
        L.mg_default_opts.argtypes = [ctypes.POINTER(mg_solve_opts)]
        L.mg_default_opts.restype = None
        L.mg_fmg_solve.argtypes = [P, ctypes.POINTER(mg_solve_opts), ctypes.POINTER(mg_solve_stats)]
        L.mg_vcycle.argtypes = [P, ctypes.POINTER(mg_solve_opts), I32,
                                ctypes.POINTER(mg_solve_stats)]
        L.mg_residual.argtypes = [P, P, P, P]
        L.mg_efield.argtypes = [P, P, P]
        L.mg_refine_scores.argtypes = [P, P]
        L.mg_regrid_plan.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I32, I64,
                                      P, P, P, P]
        L.mg_refine_near.argtypes = [P, P, P]
        L.mg_regrid_plan_near.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I32, I64,
                                           P, P, P, P]
        L.mg_transfer.argtypes = [P, P]
        L.mg_fluid_workspace_bytes.argtypes = [P, I32]
        L.mg_fluid_workspace_bytes.restype = I64
        L.mg_fluid_bind.argtypes = [P, P, I64, P, I32, ctypes.c_double]
        L.mg_fluid_stage.argtypes = [P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, P, P, P]
        L.mg_fluid_step.argtypes = [P, P, P, ctypes.c_double, I32, P]
        L.mg_step.argtypes = [P, I32, I32, I32]
        L.mg_tree_residuals.argtypes = [P, P]
        L.mg_autotune.argtypes = [P, I32, I32, P]
        L.mg_set_schedule.argtypes = [P, I32, P]
        L.mg_set_fusion.argtypes = [P, I32]
        L.mg_timing_enable.argtypes = [P, I32]
        L.mg_timing_read.argtypes = [P, ctypes.POINTER(mg_kernel_timing_t)]
        L.mg_stream_copy.argtypes = [P, P, I64, I32, P]
        L.mg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class MGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODES.get(code, code)}: {msg}")
        self.code = code
        self.name = CODES.get(code, str(code))


def check(rc):
    if rc != MG_OK:
        raise MGError(rc, lib().mg_last_error().decode())
    return rc


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------- C-named calls

def mg_tree_create(dom, level, ijk, tree=None):
    level = np.ascontiguousarray(level, dtype=np.int32)
    ijk = np.ascontiguousarray(np.asarray(ijk).reshape(-1, 3), dtype=np.int32)
    tree = None if tree is None else np.ascontiguousarray(tree, dtype=np.int32)
    h = ctypes.c_void_p()
    check(lib().mg_tree_create(ctypes.byref(h), ctypes.byref(dom), len(level), _p(level), _p(ijk),
                               None if tree is None else _p(tree)))
    return h


def mg_tree_destroy(h):
    check(lib().mg_tree_destroy(h))


def mg_tree_info(h):
    info = mg_tree_info_t()
    check(lib().mg_tree_info(h, ctypes.byref(info)))
    return info


def mg_tree_bind(h, ws_ptr, ws_bytes, stream_ptr):
    check(lib().mg_tree_bind(h, ctypes.c_void_p(ws_ptr), int(ws_bytes), ctypes.c_void_p(stream_ptr)))


def mg_tree_index(h, what, n):
    out = np.zeros(n * _WIDTH[what], dtype=np.int32)
    check(lib().mg_tree_index(h, what, _p(out)))
    return out.reshape(n, _WIDTH[what]) if _WIDTH[what] > 1 else out


def mg_field_set(h, which, dev_ptr):
    check(lib().mg_field_set(h, which, ctypes.c_void_p(dev_ptr)))


def mg_field_get(h, which, dev_ptr):
    check(lib().mg_field_get(h, which, ctypes.c_void_p(dev_ptr)))


def mg_field(h, which, dtype, nlev=None):
    """Borrowed device pointer to a field's own storage (colour-split cell
    order), its element count and, if nlev is given, the first box of each
    level (nlev + 1 entries)."""
    ptr = ctypes.c_void_p()
    n = ctypes.c_int64()
    lo = (ctypes.c_int64 * (nlev + 1))() if nlev is not None else None
    check(lib().mg_field(h, int(which), int(dtype), ctypes.byref(ptr), ctypes.byref(n),
                         None if lo is None else ctypes.cast(lo, ctypes.c_void_p)))
    return ptr.value, n.value, (list(lo) if lo is not None else None)


def mg_default_opts():
    o = mg_solve_opts()
    lib().mg_default_opts(ctypes.byref(o))
    return o


def mg_fmg_solve(h, opts, raise_on_error=True):
    st = mg_solve_stats()
    rc = lib().mg_fmg_solve(h, ctypes.byref(opts), ctypes.byref(st))
    if raise_on_error:
        check(rc)
    return st


def mg_vcycle(h, opts, n_cycles, raise_on_error=True, stats=True):
    """stats=False passes no statistics record (mg_vcycle then computes no
    residual norm for n_cycles > 0 in FP64) and returns None."""
    st = mg_solve_stats() if stats else None
    rc = lib().mg_vcycle(h, ctypes.byref(opts), int(n_cycles), ctypes.byref(st) if stats else None)
    if raise_on_error:
        check(rc)
    return st


def mg_residual(h):
    rel, l2, linf = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(lib().mg_residual(h, ctypes.byref(rel), ctypes.byref(l2), ctypes.byref(linf)))
    return dict(rel=rel.value, l2=l2.value, linf=linf.value)


def mg_efield(h, face_ptr, norm_ptr):
    """Electric field of the current phi into device buffers (either 0)."""
    check(lib().mg_efield(h, ctypes.c_void_p(face_ptr or None), ctypes.c_void_p(norm_ptr or None)))


def mg_refine_scores(h, scores_ptr):
    check(lib().mg_refine_scores(h, ctypes.c_void_p(scores_ptr)))


def mg_refine_near(h, scores_ptr, near_ptr):
    check(lib().mg_refine_near(h, ctypes.c_void_p(scores_ptr), ctypes.c_void_p(near_ptr)))


def mg_regrid_plan(h, scores, c3, deref, max_level, h_deref=float("inf")):
    """New box list (level, ijk, tree) from host scores [n][27]."""
    return _plan(lib().mg_regrid_plan, h, scores, c3, deref, max_level, h_deref)


def mg_regrid_plan_near(h, near, c3, deref, max_level, h_deref=float("inf")):
    """The same box list from host per-box values near [n] (mg_refine_near)."""
    return _plan(lib().mg_regrid_plan_near, h, near, c3, deref, max_level, h_deref)


def _plan(fn, h, values, c3, deref, max_level, h_deref):
    sc = np.ascontiguousarray(values, dtype=np.float64)
    need = ctypes.c_int64()
    args = (float(c3), float(deref), float(h_deref), int(max_level))
    n = 2 * len(sc) + 4096                   # enough unless the step refines most boxes
    while True:
        lv = np.zeros(n, dtype=np.int32)
        ij = np.zeros((n, 3), dtype=np.int32)
        tr = np.zeros(n, dtype=np.int32)
        rc = fn(h, _p(sc), *args, n, _p(lv), _p(ij), _p(tr), ctypes.byref(need))
        if rc == MG_ENOMEM and need.value > n:
            n = need.value
            continue
        check(rc)
        m = need.value
        return lv[:m], ij[:m], tr[:m]


def mg_fluid_workspace_bytes(h, n_table):
    n = lib().mg_fluid_workspace_bytes(h, int(n_table))
    if n < 0:
        check(MG_EINVAL)
    return n


def mg_fluid_bind(h, ws_ptr, ws_bytes, table, e_max):
    tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 3)
    check(lib().mg_fluid_bind(h, ctypes.c_void_p(ws_ptr), int(ws_bytes), _p(tab), len(tab), float(e_max)))


def mg_fluid_stage(h, ef_ptr, en_ptr, ne_ptr, ni_ptr, n0e_ptr, n0i_ptr, dt, wa, wb, oute_ptr, outi_ptr,
                   want_limit=True):
    lim = ctypes.c_double()
    V = ctypes.c_void_p
    check(lib().mg_fluid_stage(h, V(ef_ptr), V(en_ptr), V(ne_ptr), V(ni_ptr), V(n0e_ptr), V(n0i_ptr),
                               float(dt), float(wa), float(wb), V(oute_ptr), V(outi_ptr),
                               ctypes.byref(lim) if want_limit else None))
    return lim.value if want_limit else None


def mg_fluid_step(h, ne_ptr, ni_ptr, dt, n_vcycles=2):
    nxt = ctypes.c_double()
    check(lib().mg_fluid_step(h, ctypes.c_void_p(ne_ptr), ctypes.c_void_p(ni_ptr), float(dt),
                              int(n_vcycles), ctypes.byref(nxt)))
    return nxt.value


def mg_transfer(h_from, h_to):
    check(lib().mg_transfer(h_from, h_to))


def mg_tree_residuals(h, ntree):
    out = np.zeros(ntree)
    check(lib().mg_tree_residuals(h, _p(out)))
    return out


def mg_step(h, op, level=0, arg=0):
    check(lib().mg_step(h, op, level, arg))


def mg_autotune(h, precision, reps, n_levels):
    out = np.zeros(n_levels, dtype=np.int32)
    check(lib().mg_autotune(h, precision, reps, _p(out)))
    return out


def mg_set_fusion(h, flags):
    check(lib().mg_set_fusion(h, int(flags)))


def mg_set_schedule(h, precision, schedule):
    sch = np.ascontiguousarray(schedule, dtype=np.int32)
    check(lib().mg_set_schedule(h, precision, _p(sch)))


def mg_timing_enable(h, enable):
    check(lib().mg_timing_enable(h, int(bool(enable))))


def mg_timing_read(h):
    out = mg_kernel_timing_t()
    check(lib().mg_timing_read(h, ctypes.byref(out)))
    return dict(launches=out.launches, total_ms=out.total_ms, alg_bytes=out.alg_bytes,
                level_launches=list(out.level_launches), level_ms=list(out.level_ms),
                level_bytes=list(out.level_bytes))


def mg_stream_copy(dst_ptr, src_ptr, nbytes, blocks=0, stream_ptr=0):
    check(lib().mg_stream_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes),
                               int(blocks), ctypes.c_void_p(stream_ptr)))


# --------------------------------------------------------- convenience

def make_domain(lo=(0.0, 0.0, 0.0), length=1.0, bc_type=(0,) * 6, bc_val=(0.0,) * 6,
                per_cell_bc=False):
    d = mg_domain()
    for a in range(3):
        d.lo[a] = lo[a]
    d.len = length
    for f in range(6):
        d.bc_type[f] = int(bc_type[f])
        d.bc_val[f] = float(bc_val[f])
    d.per_cell_bc = int(bool(per_cell_bc))
    return d


class Tree:
    """An octree bound to a torch-allocated device workspace.

    Fields cross the boundary as torch float64 tensors [n, 8, 8, 8] in
    canonical box order (natural [k][j][i] layout)."""

    def __init__(self, level, ijk, tree=None, lo=(0.0, 0.0, 0.0), length=1.0,
                 bc_type=(0,) * 6, bc_val=(0.0,) * 6, per_cell_bc=False, device="cuda",
                 stream=None, bind=True):
        self.dom = make_domain(lo, length, bc_type, bc_val, per_cell_bc)
        self.h = mg_tree_create(self.dom, level, ijk, tree)
        self.info = mg_tree_info(self.h)
        self.n = int(self.info.n_boxes)
        self.nlev = int(self.info.n_levels)
        self.length = float(length)
        self.ws = None
        if bind:
            self.bind(device, stream)

    def bind(self, device="cuda", stream=None):
        """Allocate the device workspace with torch and attach it
        (mg_tree_bind: table upload and zeroed fields, waited for)."""
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # rounded up (64 MiB for large trees): trees of a mesh adaptation
        # differ by a few boxes, and equal sizes let torch's caching
        # allocator hand a freed workspace to the next tree instead of
        # making a new allocation
        need = int(self.info.workspace_bytes)
        r = _WS_ROUND if need >= 4 * _WS_ROUND else 2 << 20
        nbytes = -(-need // r) * r
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        mg_tree_bind(self.h, self.ws.data_ptr(), self.ws.numel(), self.stream.cuda_stream)

    @classmethod
    def from_workload(cls, w, **kw):
        b = w.boxes
        return cls(b.level, b.ijk, b.tree, w.lo, w.length, w.bc_type, w.bc_val, **kw)

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "h", None)
        if not h:
            return
        self.h = None
        if _finalizing():
            return  # process exit releases everything; module globals may already be gone
        mg_tree_destroy(h)

    def index(self, what):
        return mg_tree_index(self.h, what, self.n)

    def leaf_mask(self):
        return self.index(MG_IDX_CHILD)[:, 0] < 0

    def set_field(self, which, x):
        import torch
        t = torch.as_tensor(x, dtype=torch.float64)
        t = t.to(self.device).contiguous()
        if which == MG_FIELD_BCVAL:
            assert t.numel() == self.n * 6 * 64
        else:
            assert t.numel() == self.n * 512
        mg_field_set(self.h, which, t.data_ptr())
        self._keep = t  # the copy is asynchronous on the bound stream
        return t

    def get_field(self, which, to_numpy=True):
        import torch
        out = torch.empty((self.n, 8, 8, 8), dtype=torch.float64, device=self.device)
        mg_field_get(self.h, which, out.data_ptr())
        if to_numpy:
            self.stream.synchronize()
            return out.cpu().numpy()
        return out

    def set_rhs_from(self, w):
        lv, ij = self.index(MG_IDX_LEVEL), self.index(MG_IDX_IJK)
        self.set_field(MG_FIELD_RHS, w.rhs(lv, ij, self.index(MG_IDX_TREE)))

    def opts(self, **kw):
        o = mg_default_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def fmg_solve(self, **kw):
        return mg_fmg_solve(self.h, self.opts(**kw)).as_dict()

    def vcycles(self, n, **kw):
        return mg_vcycle(self.h, self.opts(**kw), n).as_dict()

    def residual(self):
        return mg_residual(self.h)

    def refine_scores(self):
        """[n][27] refinement scores (mg_refine_scores), as a numpy array."""
        import torch
        out = torch.empty((self.n, 27), dtype=torch.float64, device=self.device)
        mg_refine_scores(self.h, out.data_ptr())
        self.stream.synchronize()
        return out.cpu().numpy()

    def refine_near(self):
        """[n] per-box values of the refinement criterion with its 3-cell
        buffer (mg_refine_scores, then mg_refine_near on the GPU), as a numpy
        array: the input of mg_regrid_plan_near."""
        import torch
        sc = torch.empty((self.n, 27), dtype=torch.float64, device=self.device)
        near = torch.empty(self.n, dtype=torch.float64, device=self.device)
        mg_refine_scores(self.h, sc.data_ptr())
        mg_refine_near(self.h, sc.data_ptr(), near.data_ptr())
        self.stream.synchronize()
        return near.cpu().numpy()

    def efield(self, to_numpy=True):
        """Face components [n][3][9][8][8] and cell-centre strength [n][8][8][8]
        of E = -grad phi (mg_efield)."""
        import torch
        face = torch.empty((self.n, 3, 9, 8, 8), dtype=torch.float64, device=self.device)
        norm = torch.empty((self.n, 8, 8, 8), dtype=torch.float64, device=self.device)
        mg_efield(self.h, face.data_ptr(), norm.data_ptr())
        if to_numpy:
            self.stream.synchronize()
            return face.cpu().numpy(), norm.cpu().numpy()
        return face, norm

    def fluid_bind(self, table, e_max):
        """Allocate and attach the fluid workspace with this transport table."""
        import torch
        nb = mg_fluid_workspace_bytes(self.h, len(np.asarray(table).reshape(-1, 3)))
        self.fws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.fws.data_ptr() + 255) // 256 * 256
        mg_fluid_bind(self.h, ptr, nb, table, e_max)

    def tree_rel(self):
        return mg_tree_residuals(self.h, int(self.info.n_trees))

    def step(self, op, level=0, arg=0):
        mg_step(self.h, op, level, arg)
