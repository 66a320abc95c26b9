"""Python binding of the HIP HAPOD library (``libhapod.so``, gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/hapod.h``.  Functions carry the
C names.  Matrices are column-major: a torch tensor ``S`` of shape (n, m) with
``S.stride(0) == 1`` and leading dimension ``S.stride(1) >= n`` (for example
``torch.empty(m, n).t()``); :func:`colmajor` allocates one.  Device tensors
supply device pointers, torch's current stream is the HIP stream.

Importing this module loads the library and raises if it is missing: there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys as _sys

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhapod.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
ROUTES = {0: "passthrough", 1: "snapshots", 2: "qr", 3: "sketch", 4: "full_leaf"}
_SKETCH_KINDS = {"sparse_sign": 0, "gaussian": 1}
_SKETCH_NAMES = {v: k for k, v in _SKETCH_KINDS.items()}
_LEAF_LAYOUTS = {"column": 0, "blocks": 1}
ROW_BLOCK = 128  # rows per block of the library's row-block layout
STATUS = {0: "OK", 1: "E_INVALID", 2: "E_TREE", 3: "E_NOMEM", 4: "E_DEVICE", 5: "E_NUMERIC",
          6: "E_STATE", 7: "E_CALLBACK", 8: "E_UNSUPPORTED"}
HAPOD_EIG_MAX = 8192

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1607_05210_amd/build.py`")
_lib = C.CDLL(LIB_PATH)

_i32, _i64, _dbl, _vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
_pi64, _pdbl, _pi32 = C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int32)


class HapodTree(C.Structure):
    _fields_ = [("num_nodes", _i32), ("parent", _pi32), ("leaf_cols", _pi64), ("n", _i64),
                ("leaf_rows", _pi64)]


class HapodOptions(C.Structure):
    _fields_ = [("prec", _i32), ("reorth", _i32), ("mem_cap_bytes", _i64),
                ("node_eps_override", _pdbl), ("jacobi_max", _i32), ("autotune", _i32),
                ("leaf_wave", _i32), ("block_gram", _i32), ("right_vectors", _i32),
                ("qr_pod", _i32), ("sketch_cols", _i32), ("autotune_cache", C.c_char_p),
                ("graph_levels", _i32), ("sketch_kind", _i32), ("leaf_layout", _i32),
                ("leaf_passthrough", _i32)]


LEAF_FN = C.CFUNCTYPE(_i32, _vp, _i32, C.POINTER(_vp), _pi64, _vp)

_SIGS = {
    "hapod_gram": [_i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp],
    "hapod_gram_noalloc": [_i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp],
    "hapod_eigh": [_i64, _vp, _i64, _vp, _vp, _i64, _pi32, _vp],
    "hapod_truncate": [_i64, _vp, _dbl, _pi64, _pdbl, _vp],
    "hapod_lift": [_i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp],
    "hapod_reorth": [_i32, _i64, _i64, _vp, _i64, _pi64, _vp],
    "hapod_node_pod": [_i32, _i64, _i64, _vp, _i64, _dbl, _i32, _vp, _i64, _pdbl, _pi64, _vp],
    "hapod_plan": [C.POINTER(HapodTree), _dbl, _dbl, C.POINTER(HapodOptions), C.POINTER(_vp)],
    "hapod_plan_query": [_vp, _pdbl, _pi32, _pi64],
    "hapod_run": [_vp, LEAF_FN, _vp, _vp],
    "hapod_modes": [_vp, _i32, _vp, _i64, _pdbl, _pi64, _vp],
    "hapod_node_stats": [_vp, _pi64, _pi64, _pdbl, _pdbl],
    "hapod_right_vectors": [_vp, _vp, _i64, _vp],
    "hapod_node_pod_qr": [_i64, _i64, _vp, _i64, C.c_double, _i32, _vp, _i64, _pdbl, _pi64, _pi32, _pi32, _vp],
    "hapod_node_pod_sketch": [_i64, _i64, _vp, _i64, _dbl, _i32, _i64, C.c_uint64, _i32, _vp, _i64, _pdbl, _pi64, _pdbl,
                              _vp],
    "hapod_sketch_stats": [_vp, _i32, _pdbl],
    "hapod_plan_workspace": [_vp, _pi64, _pi64],
    "hapod_node_route": [_vp, _i32, _pi32],
    "hapod_plan_node_pod": [_vp, _i32, _vp, _i64, _i64, _vp, _i64, _pdbl, _pi64, _vp],
    "hapod_run_timing": [_vp, _pdbl],
    "hapod_plan_batch_stats": [_vp, _pi64],
    "hapod_plan_graph_stats": [_vp, _pi64, _pdbl],
    "hapod_level_timing": [_vp, _i32, _pdbl],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _i32
_lib.hapod_destroy.argtypes = [_vp]
_lib.hapod_destroy.restype = None
_lib.hapod_last_error.argtypes = []
_lib.hapod_last_error.restype = C.c_char_p

EXPORTED = sorted(list(_SIGS) + ["hapod_destroy", "hapod_last_error"])


class HapodError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.hapod_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(st, where):
    if st != 0:
        raise HapodError(st, where)


def hapod_last_error() -> str:
    return _lib.hapod_last_error().decode(errors="replace")


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def colmajor(n, m, dtype=torch.float64, device="cuda", ld=None, fill=None):
    """Column-major n x m tensor (shape (n, m), stride (1, ld))."""
    ld = n if ld is None else ld
    base = torch.empty((max(m, 0), max(ld, 1)), dtype=dtype, device=device)
    if fill is not None:
        base.fill_(fill)
    return base[:, :n].t() if n > 0 else base[:, :0].t()


def _mat(t, name, dtype=None):
    """(pointer, rows, cols, ld) of a column-major tensor."""
    if t.dim() != 2:
        raise ValueError(f"{name}: expected a 2-D tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    n, m = t.shape
    if m > 1 and n > 0 and t.stride(0) != 1:
        raise ValueError(f"{name}: must be column-major (stride(0) == 1)")
    ld = t.stride(1) if m > 1 else max(n, 1)
    return C.c_void_p(t.data_ptr()), n, m, max(ld, 1)


def to_blocks(S):
    """An n x m tensor in the library's row-block layout: a contiguous
    (ceil(n / 128), m, 128) tensor, element (r, j) at [r // 128, j, r % 128]
    (rows past n zero) -- the layout a plan made with leaf_layout="blocks"
    expects of its leaves."""
    n, m = S.shape
    nb = (n + ROW_BLOCK - 1) // ROW_BLOCK
    B = torch.zeros((nb, m, ROW_BLOCK), dtype=S.dtype, device=S.device)
    full = n // ROW_BLOCK
    if full:
        B[:full].copy_(S[:full * ROW_BLOCK].reshape(full, ROW_BLOCK, m).transpose(1, 2))
    if n > full * ROW_BLOCK:
        B[full, :, :n - full * ROW_BLOCK].copy_(S[full * ROW_BLOCK:].t())
    return B


def _blocks(t, name, dtype):
    """Pointer of a leaf in the row-block layout (see to_blocks)."""
    if t.dim() != 3 or t.shape[2] != ROW_BLOCK or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous (blocks, cols, {ROW_BLOCK}) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _elem(prec):
    return torch.float64 if prec == FP64 else torch.float32


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ---------------------------------------------------------------------------
# step-level entry points
# ---------------------------------------------------------------------------
def hapod_gram(prec, S, G=None, stream=None):
    prec = _prec(prec)
    p, n, m, lds = _mat(S, "S", _elem(prec))
    if G is None:
        G = colmajor(m, m, torch.float64, S.device)
    pg, _, _, ldg = _mat(G, "G", torch.float64)
    _check(_lib.hapod_gram(prec, n, m, p, lds, pg, ldg, _stream(stream)), "hapod_gram")
    return G


def hapod_gram_noalloc(prec, S, G, stream=None):
    """G = S^T S into the caller's G without any device allocation by the
    library (m <= 256); asynchronous on the stream."""
    prec = _prec(prec)
    p, n, m, lds = _mat(S, "S", _elem(prec))
    pg, _, _, ldg = _mat(G, "G", torch.float64)
    _check(_lib.hapod_gram_noalloc(prec, n, m, p, lds, pg, ldg, _stream(stream)), "hapod_gram_noalloc")
    return G


def hapod_eigh(G, stream=None):
    """Destroys G.  Returns (lambda, V, sweeps)."""
    pg, m, _, ldg = _mat(G, "G", torch.float64)
    lam = torch.empty(m, dtype=torch.float64, device=G.device)
    V = colmajor(m, m, torch.float64, G.device)
    pv, _, _, ldv = _mat(V, "V")
    sw = C.c_int32(0)
    _check(_lib.hapod_eigh(m, pg, ldg, C.c_void_p(lam.data_ptr()), pv, ldv, C.byref(sw), _stream(stream)),
           "hapod_eigh")
    return lam, V, sw.value


def hapod_truncate(lam, eps, stream=None):
    """Returns (rank, info[4])."""
    r = C.c_int64(0)
    info = (C.c_double * 4)()
    _check(_lib.hapod_truncate(lam.numel(), C.c_void_p(lam.data_ptr()), float(eps), C.byref(r), info,
                               _stream(stream)), "hapod_truncate")
    return r.value, list(info)


def hapod_lift(prec, S, V, N, lam=None, out=None, stream=None):
    prec = _prec(prec)
    ps, n, m, lds = _mat(S, "S", _elem(prec))
    pv, mv, _, ldv = _mat(V, "V", torch.float64)
    if out is None:
        out = colmajor(n, N, _elem(prec), S.device)
    po, _, _, ldo = _mat(out, "out", _elem(prec))
    pl = C.c_void_p(lam.data_ptr()) if lam is not None else None
    _check(_lib.hapod_lift(prec, n, m, N, ps, lds, pv, ldv, pl, po, ldo, _stream(stream)), "hapod_lift")
    return out


def hapod_reorth(prec, U, stream=None):
    prec = _prec(prec)
    pu, n, N, ldu = _mat(U, "U", _elem(prec))
    bad = C.c_int64(0)
    _check(_lib.hapod_reorth(prec, n, N, pu, ldu, C.byref(bad), _stream(stream)), "hapod_reorth")
    return bad.value


def hapod_node_pod(prec, S, eps, scaled=False, out=None, stream=None):
    """Returns (sigma[rank] numpy, out[:, :rank])."""
    import numpy as np
    prec = _prec(prec)
    ps, n, m, lds = _mat(S, "S", _elem(prec))
    if out is None:
        out = colmajor(n, m, _elem(prec), S.device)
    po, _, _, ldo = _mat(out, "out", _elem(prec))
    sig = np.zeros(max(m, 1))
    r = C.c_int64(0)
    _check(_lib.hapod_node_pod(prec, n, m, ps, lds, float(eps), int(bool(scaled)), po, ldo,
                               sig.ctypes.data_as(_pdbl), C.byref(r), _stream(stream)), "hapod_node_pod")
    return sig[:r.value].copy(), out[:, :r.value]


def hapod_node_pod_qr(S, eps, scaled=False, out=None, stream=None):
    """POD(S, eps) from a QR factor of S (FP64): returns (sigma[rank] numpy,
    out[:, :rank], {"passes": Cholesky-QR passes, "sweeps": Jacobi sweeps})."""
    import numpy as np
    ps, n, m, lds = _mat(S, "S", torch.float64)
    if out is None:
        out = colmajor(n, m, torch.float64, S.device)
    po, _, _, ldo = _mat(out, "out", torch.float64)
    sig = np.zeros(max(m, 1))
    r = C.c_int64(0)
    npass = C.c_int32(0)
    sw = C.c_int32(0)
    _check(_lib.hapod_node_pod_qr(n, m, ps, lds, float(eps), int(bool(scaled)), po, ldo,
                                  sig.ctypes.data_as(_pdbl), C.byref(r), C.byref(npass), C.byref(sw),
                                  _stream(stream)), "hapod_node_pod_qr")
    return sig[:r.value].copy(), out[:, :r.value], {"passes": npass.value, "sweeps": sw.value}


def hapod_node_pod_sketch(S, eps, ell, seed=0, scaled=False, out=None, stream=None, kind="sparse_sign"):
    """POD(S, eps) of a wide S by a randomized range finder with ell sketch
    columns (FP64), test matrix "sparse_sign" (Gaussian should its residual
    exceed eps^2) or "gaussian": returns (sigma[rank] numpy, out[:, :rank],
    {"residual", "passes_y", "passes_b", "sweeps", "ms", "ell", "kind"})."""
    import numpy as np
    ps, n, m, lds = _mat(S, "S", torch.float64)
    if out is None:
        out = colmajor(n, int(ell), torch.float64, S.device)
    po, _, _, ldo = _mat(out, "out", torch.float64)
    sig = np.zeros(max(int(ell), 1))
    r = C.c_int64(0)
    info = np.zeros(7)
    _check(_lib.hapod_node_pod_sketch(n, m, ps, lds, float(eps), int(bool(scaled)), int(ell), int(seed),
                                      _SKETCH_KINDS[kind], po, ldo, sig.ctypes.data_as(_pdbl), C.byref(r),
                                      info.ctypes.data_as(_pdbl), _stream(stream)), "hapod_node_pod_sketch")
    keys = ("residual", "passes_y", "passes_b", "sweeps", "ms", "ell")
    d = dict(zip(keys, info.tolist()[:6]))
    d["kind"] = _SKETCH_NAMES[int(info[6])]
    return sig[:r.value].copy(), out[:, :r.value], d


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------
class Plan:
    """Owns a ``hapod_plan_t``; ``run`` feeds device tensors as the leaves."""

    _destroy = _lib.hapod_destroy

    def __init__(self, parent, leaf_cols, n, eps_star, omega, prec="fp64", reorth=False,
                 mem_cap_bytes=0, eps_override=None, jacobi_max=0, leaf_rows=None, leaf_wave=0,
                 autotune=False, block_gram=False, right_vectors=False, qr_pod=False, sketch_cols=0,
                 autotune_cache=None, graph_levels=False, sketch_kind="sparse_sign", leaf_layout="column",
                 leaf_passthrough=False):
        import numpy as np
        self.num_nodes = len(parent)
        self.n = int(n)
        self.prec = _prec(prec)
        self._layout = _LEAF_LAYOUTS[leaf_layout]
        self._parent = (C.c_int32 * self.num_nodes)(*[int(p) for p in parent])
        self._cols = (C.c_int64 * self.num_nodes)(*[int(c) for c in leaf_cols])
        self._rows = None
        if leaf_rows is not None:
            self._rows = (C.c_int64 * self.num_nodes)(*[int(r) for r in leaf_rows])
        tree = HapodTree(self.num_nodes, self._parent, self._cols, self.n, self._rows)
        ov = None
        if eps_override is not None:
            arr = np.asarray(eps_override, dtype=np.float64)
            ov = arr.ctypes.data_as(_pdbl)
        opts = HapodOptions(self.prec, int(bool(reorth)), int(mem_cap_bytes), ov, int(jacobi_max),
                            int(bool(autotune)), int(leaf_wave), int(bool(block_gram)),
                            int(bool(right_vectors)), int(bool(qr_pod)), int(sketch_cols),
                            os.fsencode(autotune_cache) if autotune_cache else None, int(bool(graph_levels)),
                            _SKETCH_KINDS[sketch_kind], _LEAF_LAYOUTS[leaf_layout], int(bool(leaf_passthrough)))
        h = C.c_void_p()
        _check(_lib.hapod_plan(C.byref(tree), float(eps_star), float(omega), C.byref(opts), C.byref(h)),
               "hapod_plan")
        self._h = h
        self._keep = []

    def __del__(self):
        # no HIP calls while the interpreter shuts down: the device memory a
        # plan still holds goes back with the process
        if _sys.is_finalizing():
            return
        self.close()

    def close(self):
        """Return the plan's device memory now (``hapod_destroy``)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            Plan._destroy(h)
        self._h = None

    def query(self):
        import numpy as np
        eps = np.zeros(self.num_nodes)
        lev = np.zeros(self.num_nodes, dtype=np.int32)
        acc = np.zeros(self.num_nodes, dtype=np.int64)
        _check(_lib.hapod_plan_query(self._h, eps.ctypes.data_as(_pdbl), lev.ctypes.data_as(_pi32),
                                     acc.ctypes.data_as(_pi64)), "hapod_plan_query")
        return eps, lev, acc

    def run(self, leaves, stream=None, hold=True):
        """``leaves``: dict leaf id -> column-major device tensor (a
        ``to_blocks`` tensor when the plan has leaf_layout="blocks"), or a
        callable leaf id -> tensor (called once per leaf, in level order, just
        before the launch group that first reads it).  With ``hold`` every
        tensor handed over stays referenced until the library reports that no
        leaf given so far is read again; a provider that streams more data
        than fits passes ``hold=False`` and keeps each tensor alive itself
        until then.  A callable provider with a ``release()`` method has it
        called at that point."""
        elem = _elem(self.prec)
        held = {}
        err = []

        def cb(user, leaf, ptr, ld, s):
            try:
                if leaf < 0:
                    # release call: no leaf handed over so far is read again
                    held.clear()
                    rel = getattr(leaves, "release", None)
                    if callable(rel):
                        rel()
                    return 0
                t = leaves(leaf) if callable(leaves) else leaves[leaf]
                if self._layout == 1:
                    p, ldt = _blocks(t, f"leaf {leaf}", elem), 0
                else:
                    p, n, m, ldt = _mat(t, f"leaf {leaf}", elem)
                if hold:
                    held[leaf] = t
                ptr[0] = p.value
                ld[0] = ldt
                return 0
            except Exception as e:  # reported through HAPOD_E_CALLBACK
                err.append(e)
                return 1

        fn = LEAF_FN(cb)
        st = _lib.hapod_run(self._h, fn, None, _stream(stream))
        if st != 0 and err:
            raise HapodError(st, f"hapod_run ({err[0]!r})")
        _check(st, "hapod_run")
        return self

    def modes(self, node=-1, with_U=True, stream=None):
        import numpy as np
        r = C.c_int64(0)
        _check(_lib.hapod_modes(self._h, node, None, self.n, None, C.byref(r), _stream(stream)), "hapod_modes")
        N = r.value
        sig = np.zeros(max(N, 1))
        U = colmajor(self.n, N, _elem(self.prec)) if with_U else None
        pu = C.c_void_p(U.data_ptr()) if U is not None and N > 0 else None
        _check(_lib.hapod_modes(self._h, node, pu, self.n, sig.ctypes.data_as(_pdbl), C.byref(r),
                                _stream(stream)), "hapod_modes")
        return sig[:N].copy(), U

    def right_vectors(self, stream=None):
        """W of the factorisation S ~ U diag(sigma) W^T (Rem. 3.8, Def. 3.9):
        float64 device tensor, one row per snapshot (leaves in ascending node
        id, each leaf's columns in order), one column per root mode."""
        r = C.c_int64(0)
        _check(_lib.hapod_modes(self._h, -1, None, self.n, None, C.byref(r), None), "hapod_modes")
        nr = r.value
        inner = set(int(p) for p in self._parent if int(p) >= 0)
        ns = sum(int(self._cols[a]) for a in range(self.num_nodes) if a not in inner)
        W = colmajor(max(ns, 1), nr, torch.float64)[:ns]
        if nr > 0 and ns > 0:
            _check(_lib.hapod_right_vectors(self._h, C.c_void_p(W.data_ptr()), max(ns, 1), _stream(stream)),
                   "hapod_right_vectors")
        return W

    def node_stats(self):
        import numpy as np
        k = self.num_nodes
        m_in = np.zeros(k, dtype=np.int64)
        nneg = np.zeros(k, dtype=np.int64)
        l1 = np.zeros(k)
        lmin = np.zeros(k)
        _check(_lib.hapod_node_stats(self._h, m_in.ctypes.data_as(_pi64), nneg.ctypes.data_as(_pi64),
                                     l1.ctypes.data_as(_pdbl), lmin.ctypes.data_as(_pdbl)), "hapod_node_stats")
        return dict(m_in=m_in, n_negative=nneg, lambda1=l1, lambda_min=lmin)

    def workspace(self):
        """(worst-case bytes of a run, peak bytes the pool held in the last run)."""
        w, p = C.c_int64(0), C.c_int64(0)
        _check(_lib.hapod_plan_workspace(self._h, C.byref(w), C.byref(p)), "hapod_plan_workspace")
        return w.value, p.value

    def route(self, node=-1):
        """The route node took in the last run: passthrough, snapshots, qr, sketch or full_leaf."""
        r = C.c_int32(0)
        _check(_lib.hapod_node_route(self._h, int(node), C.byref(r)), "hapod_node_route")
        return ROUTES[r.value]

    def node_pod(self, node, S, out=None, stream=None):
        """One local POD of `node` as a run computes it, on the caller's input
        columns S (rows(node) x m): returns (sigma numpy, out[:, :rank])."""
        import numpy as np
        p, n, m, lds = _mat(S, "S", _elem(self.prec))
        if out is None:
            out = colmajor(n, m, _elem(self.prec), S.device)
        po, _, _, ldo = _mat(out, "out", _elem(self.prec))
        sig = np.zeros(max(m, 1))
        r = C.c_int64(0)
        _check(_lib.hapod_plan_node_pod(self._h, int(node), p, lds, m, po, ldo, sig.ctypes.data_as(_pdbl),
                                        C.byref(r), _stream(stream)), "hapod_plan_node_pod")
        return sig[:r.value].copy(), out[:, :r.value]

    def sketch_stats(self, node=-1):
        """Diagnostics of a node that took the sketched route (dict), or None."""
        out = (C.c_double * 13)()
        st = _lib.hapod_sketch_stats(self._h, int(node), out)
        if st == 6:
            return None
        _check(st, "hapod_sketch_stats")
        v = list(out)
        return dict(ell=int(v[0]), residual=v[1], passes_y=int(v[2]), passes_b=int(v[3]), sweeps=int(v[4]),
                    ms=dict(zip(["sketch", "orth", "cross", "residual", "small_svd", "lift"], v[5:11])),
                    kind=_SKETCH_NAMES[int(v[11])], res_cols=int(v[12]))

    def ranks(self):
        import numpy as np
        out = np.zeros(self.num_nodes, dtype=np.int64)
        for a in range(self.num_nodes):
            r = C.c_int64(0)
            _check(_lib.hapod_modes(self._h, a, None, self.n, None, C.byref(r), None), "hapod_modes")
            out[a] = r.value
        return out

    def level_timing(self, level):
        t = (C.c_double * 4)()
        _check(_lib.hapod_level_timing(self._h, int(level), t), "hapod_level_timing")
        return dict(zip(["gram", "eig", "truncate", "lift"], list(t)))

    def timing(self):
        t = (C.c_double * 6)()
        _check(_lib.hapod_run_timing(self._h, t), "hapod_run_timing")
        return dict(zip(["total", "gram", "eig", "truncate", "lift", "reorth"], list(t)))

    def graph_stats(self):
        """hipGraphs of the last run: batches captured, replayed, and the
        device time (ms) of their launches (hapod_plan_graph_stats)."""
        t = (C.c_int64 * 2)()
        ms = C.c_double(0.0)
        _check(_lib.hapod_plan_graph_stats(self._h, t, C.byref(ms)), "hapod_plan_graph_stats")
        return dict(captures=t[0], replays=t[1], ms=ms.value)

    def batch_stats(self):
        """Batches of the last run: device-driven, with ranks read back
        before the lift, device-driven ones run again (hapod_plan_batch_stats)."""
        t = (C.c_int64 * 3)()
        _check(_lib.hapod_plan_batch_stats(self._h, t), "hapod_plan_batch_stats")
        return dict(zip(["device", "host", "reruns"], list(t)))


def hapod_plan(parent, leaf_cols, n, eps_star, omega, **kw) -> Plan:
    return Plan(parent, leaf_cols, n, eps_star, omega, **kw)
