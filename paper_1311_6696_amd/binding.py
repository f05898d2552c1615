"""ctypes binding of libpepsenv (include/peps_env.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (CUDA/ROCm tensors) and the stream.
The library must have been built (``paper_1311_6696_amd.build``); loading
fails loudly otherwise.
"""
import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpepsenv.so")

PEPS_F64, PEPS_F32, PEPS_BF16 = 0, 1, 2
DTYPES = {"f64": PEPS_F64, "f32": PEPS_F32, "bf16": PEPS_BF16}
STATUS = {0: "OK", -1: "INVALID", -2: "OOM", -3: "HIP", -4: "NOT_CONVERGED", -5: "NONFINITE", -6: "UNSUPPORTED"}
OPTS_PER_STATE = 1   # peps_env_opts.flags: one options record per state
OPTS_COLUMNS = 2     # peps_env_opts.flags: also the left/right boundaries (vertical bonds from column sandwiches)
OPTS_STRICT = 4      # peps_env_opts.flags: an ALS row that reaches max_halfsweeps before tol fails the call
DEFAULT_SEED = 0x13116696
TILES = ("64x64", "128x32", "256x16", "32x128", "64x32", "64x16", "128x48", "64x80",
         "skinny16", "skinny32", "skinny48", "skinny64", "skinny80", "ketbra16", "ketbra32", "tworow")
N_STATS = 3 * 2 * len(TILES)


def variant_name(i):
    """Kernel variant of statistics slot i (see peps_ctx_profile)."""
    prec = ("f64", "f32", "bf16")[i // (2 * len(TILES))]
    out = ("f64", "f32")[(i // len(TILES)) % 2]
    tile = TILES[i % len(TILES)]
    if tile.startswith("skinny"):
        return f"tcs_kernel<{prec}, out={out}, N<={tile[6:]}>"
    if tile.startswith("ketbra"):
        return f"kb_kernel<{prec}, out={out}, dr*p<={tile[6:]}>"
    if tile == "tworow":
        return "k2_kernel (fused two-row column step, f64)"
    return f"tc_kernel<{prec}, out={out}, {tile}>"


class PepsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class State(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("phys", C.c_int32),
                ("dims", C.POINTER(C.c_int32)), ("site", C.POINTER(C.c_void_p))]


class Opts(C.Structure):
    _fields_ = [("chi", C.c_int32), ("dtype", C.c_int32), ("halfsweeps", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64), ("max_halfsweeps", C.c_int32),
                ("reserved", C.c_int32), ("tol", C.c_double)]


class Window(C.Structure):
    _fields_ = [("state", C.c_int32), ("r0", C.c_int32), ("r1", C.c_int32), ("c0", C.c_int32),
                ("c1", C.c_int32), ("ci", C.c_int32), ("cj", C.c_int32)]


class QrBlock(C.Structure):
    _fields_ = [("a", C.c_void_p), ("a_rs", C.c_int64), ("a_cs", C.c_int64),
                ("q", C.c_void_p), ("q_rs", C.c_int64), ("q_cs", C.c_int64),
                ("r", C.c_void_p), ("r_rs", C.c_int64), ("r_cs", C.c_int64),
                ("m", C.c_int32), ("n", C.c_int32)]


class SiteReq(C.Structure):
    _fields_ = [("env", C.c_void_p), ("r", C.c_int32), ("c", C.c_int32), ("dir", C.c_int32), ("n", C.c_void_p),
                ("log_z", C.c_double), ("sign", C.c_double)]


class BondReq(C.Structure):
    _fields_ = [("env", C.c_void_p), ("r", C.c_int32), ("c", C.c_int32), ("dir", C.c_int32), ("gate", C.c_void_p),
                ("b_left", C.c_void_p), ("b_right", C.c_void_p)]


class FitReq(C.Structure):
    _fields_ = [("env", C.c_void_p), ("r", C.c_int32), ("c", C.c_int32), ("dir", C.c_int32), ("gate", C.c_void_p),
                ("s1", C.c_void_p), ("s2", C.c_void_p), ("n1", C.c_void_p), ("b1", C.c_void_p),
                ("n2", C.c_void_p), ("b2", C.c_void_p)]


class OverlapReq(C.Structure):
    _fields_ = [("env_a", C.c_void_p), ("env_b", C.c_void_p), ("side", C.c_int32), ("k", C.c_int32),
                ("xy", C.c_double), ("xx", C.c_double), ("yy", C.c_double)]


class Result(C.Structure):
    _fields_ = [("log_norm", C.c_double), ("norm_sign", C.c_double), ("sz", C.POINTER(C.c_double)),
                ("bond", C.POINTER(C.c_double)), ("flops", C.c_double)]


SYMBOLS = ("peps_ctx_create", "peps_ctx_destroy", "peps_env_boundary", "peps_cluster_env", "peps_expect",
           "peps_env_free", "peps_env_info", "peps_ctx_profile", "peps_ctx_graphs", "peps_ctx_autotune",
           "peps_ctx_stats", "peps_ctx_set_workspace", "peps_qr", "peps_site_env",
           "peps_bond_env", "peps_bond_fit", "peps_boundary_overlap", "peps_qr_noalloc", "peps_env_mps",
           "peps_last_error")

_lib = None


def load(path=None):
    """Load the HIP library (once); raises OSError if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"{p} not found: build it with `python -m paper_1311_6696_amd.build`")
    lib = C.CDLL(p)
    vp, i32, pp = C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)
    lib.peps_ctx_create.argtypes = [i32, vp, pp]
    lib.peps_ctx_destroy.argtypes = [vp]
    lib.peps_ctx_destroy.restype = None
    lib.peps_env_boundary.argtypes = [vp, C.POINTER(State), i32, C.POINTER(Opts), pp]
    lib.peps_cluster_env.argtypes = [vp, C.POINTER(State), i32, C.POINTER(Window), i32, C.POINTER(Opts), pp]
    lib.peps_expect.argtypes = [vp, pp, i32, C.POINTER(Result)]
    lib.peps_env_free.argtypes = [vp]
    lib.peps_env_free.restype = None
    lib.peps_env_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_double), C.POINTER(i32),
                                  C.POINTER(i32)]
    lib.peps_ctx_profile.argtypes = [vp, i32]
    lib.peps_ctx_stats.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]
    lib.peps_ctx_set_workspace.argtypes = [vp, C.c_uint64]
    lib.peps_ctx_graphs.argtypes = [vp, C.c_int32]
    lib.peps_ctx_autotune.argtypes = [vp, C.c_int32]
    lib.peps_qr.argtypes = [vp, C.POINTER(QrBlock), i32]
    lib.peps_qr_noalloc.argtypes = [vp, C.POINTER(QrBlock), i32]
    lib.peps_env_mps.argtypes = [vp, i32, i32, i32, C.POINTER(i32), vp, C.POINTER(C.c_double)]
    lib.peps_site_env.argtypes = [vp, C.POINTER(SiteReq), i32, C.POINTER(C.c_double)]
    lib.peps_bond_env.argtypes = [vp, C.POINTER(BondReq), i32, C.POINTER(C.c_double)]
    lib.peps_boundary_overlap.argtypes = [vp, C.POINTER(OverlapReq), i32]
    lib.peps_bond_fit.argtypes = [vp, C.POINTER(FitReq), i32, C.POINTER(C.c_double)]
    lib.peps_last_error.argtypes = []
    lib.peps_last_error.restype = C.c_char_p
    for name in ("peps_ctx_create", "peps_env_boundary", "peps_cluster_env", "peps_expect", "peps_env_info",
                 "peps_ctx_profile", "peps_ctx_graphs", "peps_ctx_autotune", "peps_ctx_stats",
                 "peps_ctx_set_workspace", "peps_qr", "peps_qr_noalloc", "peps_env_mps", "peps_site_env", "peps_bond_env",
                 "peps_boundary_overlap", "peps_bond_fit"):
        getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _check(lib, code):
    if code != 0:
        raise PepsError(code, lib.peps_last_error().decode())


class RawState:
    """A lattice given as device pointers: ``ptrs[r][c]`` and ``shapes[r][c]``
    (d, Dl, Du, Dr, Dd).  Keeps the ctypes arrays alive."""

    def __init__(self, ptrs, shapes, keep=None):
        self.keep = keep   # the tensors the pointers belong to, kept alive
        self.rows, self.cols = len(ptrs), len(ptrs[0])
        flat_dims = [int(x) for row in shapes for s in row for x in s]
        self.dims = (C.c_int32 * len(flat_dims))(*flat_dims)
        flat_ptrs = [int(p) for row in ptrs for p in row]
        self.site = (C.c_void_p * len(flat_ptrs))(*flat_ptrs)
        self.phys = int(shapes[0][0][0])
        self.shapes = shapes

    def struct(self):
        return State(self.rows, self.cols, self.phys, self.dims, self.site)


class Env:
    def __init__(self, ctx, handle, rows, cols, window=False, shapes=None):
        self.ctx, self.handle, self.rows, self.cols, self.window = ctx, handle, rows, cols, window
        self.shapes = shapes   # shapes[r][c] = (d, Dl, Du, Dr, Dd) of the (window) lattice

    def site_dim(self, r, c):
        """K = Dl Du Dr Dd of site (r, c): its norm environment is K x K."""
        _, Dl, Du, Dr, Dd = self.shapes[r][c]
        return int(Dl * Du * Dr * Dd)

    def info(self, full=False):
        """Squared ALS centre norms per truncated row (top rows, then bottom
        rows) and half-sweep, NaN past a row's last; with full=True also the
        half-sweeps each row ran and the number of rows that stopped at the
        cap before the tolerance."""
        lib = self.ctx.lib
        n, h, u = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib, lib.peps_env_info(self.handle, C.byref(n), C.byref(h), None, None, C.byref(u)))
        om = (C.c_double * max(1, n.value * h.value))()
        sw = (C.c_int32 * max(1, n.value))()
        _check(lib, lib.peps_env_info(self.handle, None, None, om, sw, None))
        w = np.array(om[: n.value * h.value]).reshape(n.value, h.value)
        if full:
            return w, np.array(sw[: n.value]), u.value
        return w

    def mps(self, side, k):
        """Stored boundary after k absorbed rows from `side` (0 top, 1 bottom,
        2 left, 3 right) as (list of float64 GPU tensors [a, k, b, a'],
        log_scale)."""
        import torch
        lib = self.ctx.lib
        out, ls = [], C.c_double()
        n = self.cols if side < 2 else self.rows
        for c in range(n):
            d = (C.c_int32 * 4)()
            _check(lib, lib.peps_env_mps(self.handle, side, k, c, d, None, None))
            t = torch.empty(tuple(d), dtype=torch.float64, device="cuda")
            _check(lib, lib.peps_env_mps(self.handle, side, k, c, None, C.c_void_p(t.data_ptr()), C.byref(ls)))
            out.append(t)
        return out, ls.value

    def free(self):
        if self.handle:
            self.ctx.lib.peps_env_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A library context on one device and stream (raw pointer interface)."""

    def __init__(self, device=0, stream=0, lib=None):
        self.lib = lib or load()
        h = C.c_void_p()
        _check(self.lib, self.lib.peps_ctx_create(int(device), C.c_void_p(int(stream) or None), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            self.lib.peps_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def opts(chi, dtype="f64", halfsweeps=4, seed=DEFAULT_SEED, tol=0.0, max_halfsweeps=0):
        return Opts(int(chi), DTYPES[dtype] if isinstance(dtype, str) else int(dtype), int(halfsweeps), 0,
                    int(seed) & ((1 << 64) - 1), int(max_halfsweeps), 0, float(tol))

    def env_boundary_raw(self, states, chi, dtype="f64", halfsweeps=4, seed=DEFAULT_SEED, columns=False,
                         tol=0.0, max_halfsweeps=0, strict=False):
        """chi, halfsweeps, seed: one value for all states, or a sequence with
        one per state (passed as per-state options records).  columns: also
        the left and right boundaries (OPTS_COLUMNS).  tol > 0: ALS sweeps
        until the squared centre norm settles (at most max_halfsweeps; strict
        makes an unconverged row an error)."""
        n = len(states)
        arr = (State * n)(*[s.struct() for s in states])
        out = (C.c_void_p * n)()
        flags = (OPTS_COLUMNS if columns else 0) | (OPTS_STRICT if strict else 0)
        per = [np.ndim(x) != 0 for x in (chi, halfsweeps, seed)]
        if not any(per):
            o = self.opts(chi, dtype, halfsweeps, seed, tol, max_halfsweeps)
            o.flags = flags
            _check(self.lib, self.lib.peps_env_boundary(self.handle, arr, n, C.byref(o), out))
        else:
            vals = [list(x) if p else [x] * n for x, p in zip((chi, halfsweeps, seed), per)]
            if any(len(v) != n for v in vals):
                raise ValueError("one chi, halfsweeps or seed per state")
            recs = [self.opts(c, dtype, h, s, tol, max_halfsweeps) for c, h, s in zip(*vals)]
            for r in recs:
                r.flags = OPTS_PER_STATE | flags
            o = (Opts * n)(*recs)
            _check(self.lib, self.lib.peps_env_boundary(self.handle, arr, n, o, out))
        return [Env(self, out[i], s.rows, s.cols, shapes=s.shapes) for i, s in enumerate(states)]

    def cluster_env_raw(self, states, windows, chi, dtype="f64", halfsweeps=4, seed=DEFAULT_SEED, columns=False):
        n = len(states)
        arr = (State * n)(*[s.struct() for s in states])
        w = (Window * len(windows))(*[Window(*[int(x) for x in win]) for win in windows])
        out = (C.c_void_p * len(windows))()
        o = self.opts(chi, dtype, halfsweeps, seed)
        o.flags = OPTS_COLUMNS if columns else 0
        _check(self.lib, self.lib.peps_cluster_env(self.handle, arr, n, w, len(windows), C.byref(o), out))
        return [Env(self, out[i], win[2] - win[1] + 1, win[4] - win[3] + 1, window=True,
                    shapes=[row[win[3]: win[4] + 1] for row in states[win[0]].shapes[win[1]: win[2] + 1]])
                for i, win in enumerate(windows)]

    def expect(self, envs):
        n = len(envs)
        hs = (C.c_void_p * n)(*[e.handle for e in envs])
        bufs = []
        res = (Result * n)()
        for i, e in enumerate(envs):
            nsz = 1 if e.window else e.rows * e.cols
            nb = 2 if e.window else e.rows * (e.cols - 1) + (e.rows - 1) * e.cols
            sz = np.zeros(nsz)
            bd = np.zeros(max(nb, 1))
            bufs.append((sz, bd))
            res[i].sz = sz.ctypes.data_as(C.POINTER(C.c_double))
            res[i].bond = bd.ctypes.data_as(C.POINTER(C.c_double))
        _check(self.lib, self.lib.peps_expect(self.handle, hs, n, res))
        out = []
        for i, e in enumerate(envs):
            sz, bd = bufs[i]
            d = dict(log_norm=res[i].log_norm, sign=res[i].norm_sign, flops=res[i].flops)
            if e.window:
                d.update(sz=sz[0], right=bd[0], down=bd[1])
            else:
                R, Cc = e.rows, e.cols
                d.update(sz=sz.reshape(R, Cc), bond_h=bd[: R * (Cc - 1)].reshape(R, Cc - 1),
                         bond_v=bd[R * (Cc - 1): R * (Cc - 1) + (R - 1) * Cc].reshape(R - 1, Cc))
            out.append(d)
        return out

    def autotune(self, mode=1):
        """1: time launch shapes for new contraction signatures; 0: stop, keep
        the choices; 2: forget them."""
        _check(self.lib, self.lib.peps_ctx_autotune(self.handle, int(mode)))

    def graphs(self, enable=True):
        """Replay byte-identical launch sequences from captured HIP graphs."""
        _check(self.lib, self.lib.peps_ctx_graphs(self.handle, 1 if enable else 0))

    def profile(self, enable=True):
        _check(self.lib, self.lib.peps_ctx_profile(self.handle, 1 if enable else 0))

    def stats(self):
        """Per-variant (flops, milliseconds, launches, bytes) since profiling was enabled."""
        f = (C.c_double * N_STATS)()
        m = (C.c_double * N_STATS)()
        n = (C.c_int64 * N_STATS)()
        b = (C.c_double * N_STATS)()
        _check(self.lib, self.lib.peps_ctx_stats(self.handle, f, m, n, b))
        return np.array(f[:]), np.array(m[:]), np.array(n[:]), np.array(b[:])

    def set_workspace(self, nbytes):
        _check(self.lib, self.lib.peps_ctx_set_workspace(self.handle, int(nbytes)))

    def site_env_raw(self, reqs):
        """reqs: sequence of (env, r, c, device address of K*K doubles[, dir]).
        Returns ([(log_z, sign)], flops)."""
        arr = (SiteReq * len(reqs))(*[SiteReq(q[0].handle, int(q[1]), int(q[2]), int(q[4]) if len(q) > 4 else 0,
                                              int(q[3]), 0.0, 0.0) for q in reqs])
        fl = C.c_double()
        _check(self.lib, self.lib.peps_site_env(self.handle, arr, len(reqs), C.byref(fl)))
        return [(arr[i].log_z, arr[i].sign) for i in range(len(reqs))], fl.value

    def bond_env_raw(self, reqs):
        """reqs: sequence of (env, r, c, gate, b_left, b_right[, dir]) with
        device addresses (0 for an output not wanted).  Returns the flops."""
        arr = (BondReq * len(reqs))(*[BondReq(q[0].handle, int(q[1]), int(q[2]), int(q[6]) if len(q) > 6 else 0,
                                              int(q[3]), int(q[4]) or None, int(q[5]) or None) for q in reqs])
        fl = C.c_double()
        _check(self.lib, self.lib.peps_bond_env(self.handle, arr, len(reqs), C.byref(fl)))
        return fl.value

    def bond_fit_raw(self, reqs):
        """reqs: sequence of (env, r, c, dir, gate, s1, s2, n1, b1, n2, b2)
        with device addresses.  Returns the flops."""
        arr = (FitReq * len(reqs))(*[FitReq(q[0].handle, int(q[1]), int(q[2]), int(q[3]), *[int(p) for p in q[4:]])
                                     for q in reqs])
        fl = C.c_double()
        _check(self.lib, self.lib.peps_bond_fit(self.handle, arr, len(reqs), C.byref(fl)))
        return fl.value

    def boundary_overlap(self, reqs):
        """reqs: sequence of (env_a, env_b, side, k).  Returns [(xy, xx, yy)];
        the boundary fidelity is |xy| / sqrt(xx * yy)."""
        arr = (OverlapReq * len(reqs))(*[OverlapReq(a.handle, b.handle, int(s), int(k), 0.0, 0.0, 0.0)
                                         for a, b, s, k in reqs])
        _check(self.lib, self.lib.peps_boundary_overlap(self.handle, arr, len(reqs)))
        return [(arr[i].xy, arr[i].xx, arr[i].yy) for i in range(len(reqs))]

    def qr_raw(self, blocks, noalloc=False):
        """blocks: sequence of (a, a_rs, a_cs, q, q_rs, q_cs, r, r_rs, r_cs, m, n)
        with device addresses (r may be 0).  noalloc: peps_qr_noalloc (all
        workspace in the library's fixed per-GPU array)."""
        arr = (QrBlock * len(blocks))(*[QrBlock(*[int(v) if v is not None else None for v in b]) for b in blocks])
        fn = self.lib.peps_qr_noalloc if noalloc else self.lib.peps_qr
        _check(self.lib, fn(self.handle, arr, len(blocks)))


# ------------------------------------------------------------ torch layer ---

def to_device(A, device="cuda"):
    """Site tensors (nested lists of float64 numpy arrays) -> contiguous
    float64 torch tensors on the GPU."""
    import torch
    return [[torch.as_tensor(np.ascontiguousarray(t), dtype=torch.float64, device=device) for t in row] for row in A]


def state_of(tensors):
    """RawState from nested lists of float64 device tensors (a RawState is
    returned as it is, so a caller that calls repeatedly on the same lattice
    can marshal its pointers once)."""
    if isinstance(tensors, RawState):
        return tensors
    import torch
    f64 = torch.float64
    for row in tensors:
        for t in row:
            if t.dtype is not f64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("site tensors must be contiguous float64 GPU tensors")
    return RawState([[t.data_ptr() for t in row] for row in tensors],
                    [[tuple(t.shape) for t in row] for row in tensors], keep=tensors)


class Session:
    """Context bound to torch's current device and stream."""

    def __init__(self, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch: the HIP library needs an MI355X")
        dev = torch.cuda.current_device() if device is None else device
        self.torch = torch
        self.stream = torch.cuda.current_stream(dev)
        self.ctx = Context(dev, self.stream.cuda_stream)

    def env_boundary(self, tensors_list, chi, dtype="f64", halfsweeps=4, seed=DEFAULT_SEED, columns=False,
                     tol=0.0, max_halfsweeps=0, strict=False):
        states = [state_of(t) for t in tensors_list]
        return self.ctx.env_boundary_raw(states, chi, dtype, halfsweeps, seed, columns, tol, max_halfsweeps, strict)

    def cluster_env(self, tensors_list, windows, chi, dtype="f64", halfsweeps=4, seed=DEFAULT_SEED, columns=False):
        states = [state_of(t) for t in tensors_list]
        return self.ctx.cluster_env_raw(states, windows, chi, dtype, halfsweeps, seed, columns)

    def expect(self, envs):
        return self.ctx.expect(envs)

    def site_env(self, reqs):
        """reqs: sequence of (env, r, c[, dir]).  Returns ([(N, log_z, sign)],
        flops) with N a K x K float64 GPU tensor (ket legs (l, u, r, d) as
        rows) scaled so that sum_p A N A = sign; dir 1 takes it from the
        column sandwich."""
        torch = self.torch
        outs = [torch.empty((q[0].site_dim(q[1], q[2]),) * 2, dtype=torch.float64, device="cuda") for q in reqs]
        res, fl = self.ctx.site_env_raw([(q[0], q[1], q[2], n.data_ptr(), q[3] if len(q) > 3 else 0)
                                         for q, n in zip(reqs, outs)])
        return [(n, lz, sg) for n, (lz, sg) in zip(outs, res)], fl

    def bond_env(self, reqs):
        """reqs: sequence of (env, r, c, gate[, dir]) with gate a (d, d, d, d)
        float64 GPU tensor G[p, P, q, Q]; dir 0 the bond (r,c)-(r,c+1), dir 1
        the bond (r,c)-(r+1,c).  Returns ([(b_left, b_right)], flops), each b
        a (d, K) float64 GPU tensor of that site."""
        torch = self.torch
        outs, raw = [], []
        for q in reqs:
            e, r, c, g = q[:4]
            dr = q[4] if len(q) > 4 else 0
            if not g.is_cuda or g.dtype != torch.float64 or not g.is_contiguous():
                raise ValueError("the gate must be a contiguous float64 GPU tensor")
            d = int(e.shapes[r][c][0])
            r2, c2 = (r + 1, c) if dr == 1 else (r, c + 1)
            bl = torch.empty((d, e.site_dim(r, c)), dtype=torch.float64, device="cuda")
            br = torch.empty((d, e.site_dim(r2, c2)), dtype=torch.float64, device="cuda")
            outs.append((bl, br))
            raw.append((e, r, c, g.data_ptr(), bl.data_ptr(), br.data_ptr(), dr))
        fl = self.ctx.bond_env_raw(raw)
        return outs, fl

    def bond_fit(self, reqs):
        """reqs: sequence of (env, r, c, dir, gate, s1, s2) with float64 GPU
        tensors (s1, s2 shaped like the bond's sites).  Returns
        ([(n1, b1, n2, b2)], flops): the two local problems of fitting
        gate psi with the bond's sites replaced by s1, s2."""
        torch = self.torch
        outs, raw = [], []
        for e, r, c, dr, g, s1, s2 in reqs:
            for t in (g, s1, s2):
                if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
                    raise ValueError("gate and substitutes must be contiguous float64 GPU tensors")
            r2, c2 = (r + 1, c) if dr == 1 else (r, c + 1)
            if tuple(s1.shape) != tuple(e.shapes[r][c]) or tuple(s2.shape) != tuple(e.shapes[r2][c2]):
                raise ValueError("substitutes must have the shapes of the bond's sites")
            d = int(e.shapes[r][c][0])
            K1, K2 = e.site_dim(r, c), e.site_dim(r2, c2)
            o = (torch.empty((K1, K1), dtype=torch.float64, device="cuda"),
                 torch.empty((d, K1), dtype=torch.float64, device="cuda"),
                 torch.empty((K2, K2), dtype=torch.float64, device="cuda"),
                 torch.empty((d, K2), dtype=torch.float64, device="cuda"))
            outs.append(o)
            raw.append((e, r, c, dr, g.data_ptr(), s1.data_ptr(), s2.data_ptr()) + tuple(t.data_ptr() for t in o))
        fl = self.ctx.bond_fit_raw(raw)
        return outs, fl

    def qr(self, mats, inplace=False):
        """Thin QR (R_ii >= 0) of float64 GPU matrices (2-D tensors, any
        strides), as one batched call.  Returns [(Q, R)]; with inplace=True
        Q overwrites each input."""
        torch = self.torch
        out, blocks = [], []
        for A in mats:
            if not A.is_cuda or A.dtype != torch.float64 or A.dim() != 2:
                raise ValueError("QR blocks must be 2-D float64 GPU tensors")
            m, n = A.shape
            Q = A if inplace else torch.empty((m, n), dtype=torch.float64, device=A.device)
            R = torch.empty((n, n), dtype=torch.float64, device=A.device)
            blocks.append((A.data_ptr(), A.stride(0), A.stride(1), Q.data_ptr(), Q.stride(0), Q.stride(1),
                           R.data_ptr(), R.stride(0), R.stride(1), m, n))
            out.append((Q, R))
        self.ctx.qr_raw(blocks)
        return out
