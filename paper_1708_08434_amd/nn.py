"""ctypes binding of the learned correction step (include/mg_nn.h).

Argument marshalling only: the network's forward and backward passes, the
optimiser, the input gathering and the learned step all run in libmg's HIP
kernels.  Device buffers are torch tensors (plumbing for memory and streams).
"""
import ctypes
import sys

import numpy as np

from . import mg as M

MG_NN_PARAMS = 7809

EXPORTS = ["mg_nn_state_bytes", "mg_nn_create", "mg_nn_destroy", "mg_nn_set_params",
           "mg_nn_get_params", "mg_nn_forward", "mg_nn_train_bytes", "mg_nn_gradient",
           "mg_nn_get_grad", "mg_nn_adam", "mg_learned_bytes", "mg_nn_inputs", "mg_nn_targets",
           "mg_learned_step", "mg_learned_solve", "mg_nn_gradient_static", "mg_nn_bind",
           "mg_learned_level_step"]
MG_NN_STATIC_MAX_BOXES = 64


class mg_adam_opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class mg_learned_stats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("fallback_cycle", ctypes.c_int32),
                ("t_learned_ms", ctypes.c_double)]


_ready = False


def lib():
    global _ready
    L = M.lib()
    if not _ready:
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.mg_nn_state_bytes.argtypes = []
        L.mg_nn_state_bytes.restype = I64
        L.mg_nn_create.argtypes = [ctypes.POINTER(P), P, I64, P]
        L.mg_nn_destroy.argtypes = [P]
        L.mg_nn_set_params.argtypes = [P, P]
        L.mg_nn_get_params.argtypes = [P, P]
        L.mg_nn_forward.argtypes = [P, I64, P, P]
        L.mg_nn_train_bytes.argtypes = [I64]
        L.mg_nn_train_bytes.restype = I64
        L.mg_nn_gradient.argtypes = [P, I64, P, P, P, P, I64, P]
        L.mg_nn_gradient_static.argtypes = [P, I64, P, P, P, P]
        L.mg_nn_get_grad.argtypes = [P, P]
        L.mg_nn_adam.argtypes = [P, ctypes.POINTER(mg_adam_opts)]
        L.mg_learned_bytes.argtypes = [P]
        L.mg_learned_bytes.restype = I64
        L.mg_nn_inputs.argtypes = [P, P, P]
        L.mg_nn_targets.argtypes = [P, P, P, P]
        L.mg_learned_step.argtypes = [P, P, P, I64, P]
        L.mg_nn_bind.argtypes = [P, P, P, I64]
        L.mg_learned_level_step.argtypes = [P, P, P, I64, ctypes.c_int32, P]
        L.mg_learned_solve.argtypes = [P, P, P, I64, ctypes.POINTER(M.mg_solve_opts),
                                       ctypes.POINTER(M.mg_solve_stats),
                                       ctypes.POINTER(mg_learned_stats)]
        _ready = True
    return L


def _vp(t):
    return ctypes.c_void_p(None if t is None else t.data_ptr())


# ---------------------------------------------------------- C-named calls

def mg_nn_state_bytes():
    return int(lib().mg_nn_state_bytes())


def mg_nn_create(state_ptr, state_bytes, stream_ptr):
    h = ctypes.c_void_p()
    M.check(lib().mg_nn_create(ctypes.byref(h), ctypes.c_void_p(state_ptr), int(state_bytes),
                               ctypes.c_void_p(stream_ptr)))
    return h


def mg_nn_destroy(h):
    M.check(lib().mg_nn_destroy(h))


def mg_nn_set_params(h, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == MG_NN_PARAMS
    M.check(lib().mg_nn_set_params(h, p.ctypes.data_as(ctypes.c_void_p)))


def mg_nn_get_params(h):
    p = np.zeros(MG_NN_PARAMS, dtype=np.float32)
    M.check(lib().mg_nn_get_params(h, p.ctypes.data_as(ctypes.c_void_p)))
    return p


def mg_nn_get_grad(h):
    g = np.zeros(MG_NN_PARAMS, dtype=np.float32)
    M.check(lib().mg_nn_get_grad(h, g.ctypes.data_as(ctypes.c_void_p)))
    return g


def mg_nn_forward(h, nbox, x_ptr, y_ptr):
    M.check(lib().mg_nn_forward(h, int(nbox), ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)))


def mg_nn_train_bytes(nbox):
    return int(lib().mg_nn_train_bytes(int(nbox)))


def mg_nn_gradient(h, nbox, idx_ptr, x_ptr, t_ptr, ws_ptr, ws_bytes, want_loss=True):
    loss = ctypes.c_double()
    M.check(lib().mg_nn_gradient(h, int(nbox), ctypes.c_void_p(idx_ptr), ctypes.c_void_p(x_ptr),
                                 ctypes.c_void_p(t_ptr), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                 ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def mg_nn_gradient_static(h, nbox, idx_ptr, x_ptr, t_ptr, want_loss=True):
    """mg_nn_gradient with the library's static training buffers (no
    workspace, no allocation; nbox <= MG_NN_STATIC_MAX_BOXES)."""
    loss = ctypes.c_double()
    M.check(lib().mg_nn_gradient_static(h, int(nbox), ctypes.c_void_p(idx_ptr), ctypes.c_void_p(x_ptr),
                                        ctypes.c_void_p(t_ptr), ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def mg_nn_adam(h, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    o = mg_adam_opts(lr, beta1, beta2, eps)
    M.check(lib().mg_nn_adam(h, ctypes.byref(o)))


def mg_learned_bytes(tree_h):
    return int(lib().mg_learned_bytes(tree_h))


def mg_nn_inputs(tree_h, x_ptr, scale_ptr):
    M.check(lib().mg_nn_inputs(tree_h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(scale_ptr)))


def mg_nn_targets(tree_h, ref_ptr, scale_ptr, target_ptr):
    M.check(lib().mg_nn_targets(tree_h, ctypes.c_void_p(ref_ptr), ctypes.c_void_p(scale_ptr),
                                ctypes.c_void_p(target_ptr)))


def mg_learned_step(tree_h, nn_h, ws_ptr, ws_bytes, n_trees, n_levels):
    steps = np.zeros((n_trees, n_levels + 1))
    M.check(lib().mg_learned_step(tree_h, nn_h, ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                  steps.ctypes.data_as(ctypes.c_void_p)))
    return steps


def mg_learned_solve(tree_h, nn_h, ws_ptr, ws_bytes, opts, raise_on_error=True):
    st = M.mg_solve_stats()
    ls = mg_learned_stats()
    rc = lib().mg_learned_solve(tree_h, nn_h, ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                ctypes.byref(opts), ctypes.byref(st), ctypes.byref(ls))
    if raise_on_error:
        M.check(rc)
    return st, ls


def mg_learned_level_step(tree_h, nn_h, ws_ptr, ws_bytes, level, ntree):
    """The per-level learned step on one level of the current phi; returns
    the per-tree steps."""
    st = np.zeros(ntree)
    M.check(lib().mg_learned_level_step(tree_h, nn_h, ctypes.c_void_p(ws_ptr), int(ws_bytes), int(level),
                                        st.ctypes.data_as(ctypes.c_void_p)))
    return st


def mg_nn_bind(tree_h, nn_h, ws_ptr, ws_bytes):
    """Attach a network and its learned-step workspace to a tree for
    mg_fmg_solve(precision=MG_LEARNED) (nn_h None detaches)."""
    M.check(lib().mg_nn_bind(tree_h, nn_h, ctypes.c_void_p(ws_ptr), int(ws_bytes)))


# --------------------------------------------------------- convenience

class Net:
    """A network whose state lives in a torch-allocated device buffer."""

    def __init__(self, params=None, device="cuda", stream=None):
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = mg_nn_state_bytes()
        self.state = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.h = mg_nn_create(self.state.data_ptr(), n, self.stream.cuda_stream)
        self._ws = None
        if params is not None:
            self.set_params(params)

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "h", None)
        if not h:
            return
        self.h = None
        if _finalizing():
            return  # process exit releases everything; module globals may already be gone
        mg_nn_destroy(h)

    def set_params(self, p):
        mg_nn_set_params(self.h, p)

    def get_params(self):
        return mg_nn_get_params(self.h)

    def get_grad(self):
        return mg_nn_get_grad(self.h)

    def forward(self, x):
        import torch
        x = x.to(self.device, torch.float32).contiguous().reshape(-1, 1000)
        y = torch.empty((x.shape[0], 8, 8, 8), dtype=torch.float32, device=self.device)
        mg_nn_forward(self.h, x.shape[0], x.data_ptr(), y.data_ptr())
        return y

    def workspace(self, nbox):
        import torch
        need = mg_nn_train_bytes(nbox)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def gradient(self, x, target, idx=None, want_loss=True):
        """Loss over boxes idx (device int32 tensor, or all) and its gradient."""
        nbox = int(idx.numel()) if idx is not None else int(x.shape[0])
        ws = self.workspace(nbox)
        return mg_nn_gradient(self.h, nbox, 0 if idx is None else idx.data_ptr(), x.data_ptr(),
                              target.data_ptr(), ws.data_ptr(), ws.numel(), want_loss)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        mg_nn_adam(self.h, lr, beta1, beta2, eps)


class Learned:
    """Workspace for learned steps on one tree (mg.Tree)."""

    def __init__(self, tree):
        import torch
        self.tree = tree
        self.nleaf = int(tree.info.n_leaf_boxes)
        self.ws = torch.empty(mg_learned_bytes(tree.h), dtype=torch.uint8, device=tree.device)

    def inputs(self):
        import torch
        x = torch.empty((self.nleaf, 10, 10, 10), dtype=torch.float32, device=self.tree.device)
        s = torch.empty(self.nleaf, dtype=torch.float32, device=self.tree.device)
        mg_nn_inputs(self.tree.h, x.data_ptr(), s.data_ptr())
        return x, s

    def targets(self, ref, scale):
        import torch
        ref = ref.to(self.tree.device, torch.float64).contiguous()
        t = torch.empty((self.nleaf, 8, 8, 8), dtype=torch.float32, device=self.tree.device)
        mg_nn_targets(self.tree.h, ref.data_ptr(), scale.data_ptr(), t.data_ptr())
        return t

    def step(self, net):
        return mg_learned_step(self.tree.h, net.h, self.ws.data_ptr(), self.ws.numel(),
                               int(self.tree.info.n_trees), self.tree.nlev)

    def level_step(self, net, level):
        return mg_learned_level_step(self.tree.h, net.h, self.ws.data_ptr(), self.ws.numel(), level,
                                     int(self.tree.info.n_trees))

    def solve(self, net, raise_on_error=True, **kw):
        st, ls = mg_learned_solve(self.tree.h, net.h, self.ws.data_ptr(), self.ws.numel(),
                                  self.tree.opts(**kw), raise_on_error)
        d = st.as_dict()
        d.update(accepted=ls.accepted, fallback_cycle=ls.fallback_cycle,
                 t_learned_ms=ls.t_learned_ms)
        return d


def training_pairs(tree, states=(0, 1, 2), ref_tol=1e-11):
    """(input, target) pairs of every leaf box for the tree's current
    right-hand side: the reference is the solve to ref_tol; the states are
    the iterates after the FMG pass followed by k V-cycles."""
    import torch
    tree.fmg_solve(rel_tol=ref_tol, max_cycles=60)
    ref = tree.get_field(M.MG_FIELD_PHI, to_numpy=False)
    L = Learned(tree)
    xs, ts = [], []
    for k in states:
        tree.fmg_solve(rel_tol=1e300)
        if k:
            tree.vcycles(k)
        x, s = L.inputs()
        xs.append(x)
        ts.append(L.targets(ref, s))
    return torch.cat(xs), torch.cat(ts)


def train(net, x, target, steps=300, batch=1024, lr=1e-3, seed=0, log_every=50):
    """Adam on random mini-batches of the pairs; returns the logged losses."""
    import torch
    n = int(x.shape[0])
    batch = min(batch, n)
    rng = np.random.default_rng(seed)
    losses = []
    for k in range(steps):
        idx = torch.from_numpy(rng.choice(n, batch, replace=False).astype(np.int32)).to(net.device)
        want = log_every and (k % log_every == 0 or k == steps - 1)
        loss = net.gradient(x, target, idx=idx, want_loss=bool(want))
        if want:
            losses.append((k, loss))
        net.adam(lr)
    return losses
