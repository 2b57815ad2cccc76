"""Python binding of libnbody (MI355X direct N-body forces).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libnbody.so`` behind the C ABI of ``include/nbody.h``.  PyTorch
provides device memory and streams.  There is no CPU fallback: importing
works without a GPU (the library loads), but every compute call needs a
context on a GPU device and fails loudly otherwise.

Array convention: vector fields are float64 tensors of shape (3, n) whose
rows are the x, y, z components (each row contiguous); scalars per particle
are float64 tensors of shape (n,).  Times and steps are int64 ticks of 2^-20
time units.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = ["lib", "Context", "Hermite", "NBodyError", "PREC", "TICKS_PER_UNIT",
           "LIB_PATH", "block_level", "EXPORTS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")
TICKS_PER_UNIT = 1 << 20
PREC = {"fp32": 0, "ds": 1, "ds_comp": 1}

#: Every symbol include/nbody.h declares.
EXPORTS = [
    "nbody_abi_version", "nbody_create", "nbody_destroy", "nbody_reserve", "nbody_sync",
    "nbody_last_error", "nbody_set_tile", "nbody_get_tile", "nbody_autotune", "nbody_force",
    "nbody_select_active", "nbody_hermite_create", "nbody_hermite_destroy",
    "nbody_hermite_set_state", "nbody_hermite_get_state", "nbody_hermite_step",
    "nbody_hermite_advance", "nbody_hermite_energy", "nbody_hermite_state_bytes",
    "nbody_hermite_save", "nbody_hermite_load", "nbody_block_level", "nbody_kernel_timing",
    "nbody_kernel_time", "nbody_force_vjp", "nbody_force_vjp_self", "nbody_shared_ckpt_bytes",
    "nbody_shared_run", "nbody_shared_adjoint", "nbody_force_batched", "nbody_batch_hermite",
    "nbody_autotune_batched", "nbody_force_acc", "nbody_force_nn", "nbody_leapfrog",
    "nbody_force_noalloc",
]

#: The GRAPE-6-style interface (include/nbody_grape.h).
GRAPE_EXPORTS = [
    "GPU_open", "GPU_close", "GPU_npipes", "GPU_set_j_particle", "GPU_set_ti", "GPUcalc_firsthalf",
    "GPUcalc_lasthalf", "GPUcalc_lasthalf2", "GPU_set_nn", "GPU_set_precision", "GPU_last_error",
]

ERRORS = {0: "OK", -1: "NBODY_ERR_ARG", -2: "NBODY_ERR_NOMEM", -3: "NBODY_ERR_DEVICE",
          -4: "NBODY_ERR_UNSUPPORTED", -5: "NBODY_ERR_STATE"}


class NBodyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Src(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]


class Out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ax", "ay", "az", "jx", "jy", "jz", "pot")]


class Tile(C.Structure):
    _fields_ = [("tile_j", C.c_int), ("ipt", C.c_int), ("wg", C.c_int), ("split", C.c_int),
                ("jsrc", C.c_int), ("unroll", C.c_int), ("waves", C.c_int)]

    def as_dict(self):
        return {"tile_j": self.tile_j, "ipt": self.ipt, "wg": self.wg, "split": self.split,
                "jsrc": self.jsrc, "unroll": self.unroll, "waves": self.waves}


class HermiteOpts(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("eta", C.c_double),
                ("eta_start", C.c_double), ("dt_min_log2", C.c_int), ("dt_max_log2", C.c_int),
                ("shared_dt_log2", C.c_int), ("prec", C.c_int)]


class HermiteStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("sum_active", C.c_int64), ("t_ticks", C.c_int64)]


_lib = None


def lib():
    """Load libnbody.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0707_0438_amd.build`")
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
    # first makes libnbody bind to that same runtime instead of a second copy
    # from the system ROCm, so tensors and streams are shared by one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "nbody_abi_version": ([], I),
        "nbody_create": ([C.POINTER(P), I, C.c_char_p], I),
        "nbody_destroy": ([P], I),
        "nbody_reserve": ([P, I64, I64], I),
        "nbody_sync": ([P, P], I),
        "nbody_last_error": ([P], C.c_char_p),
        "nbody_set_tile": ([P, I, C.POINTER(Tile)], I),
        "nbody_get_tile": ([P, I, I64, I64, C.POINTER(Tile)], I),
        "nbody_autotune": ([P, P, I, D, D, I64, Src, I64, Src, Out, I, C.POINTER(Tile),
                            C.POINTER(D)], I),
        "nbody_force": ([P, P, I, D, D, I64, Src, P, I64, Src, Out], I),
        "nbody_force_noalloc": ([P, P, I, D, D, I64, Src, P, I64, Src, Out], I),
        "nbody_select_active": ([P, P, I64, P, P, P, C.POINTER(I64), C.POINTER(I64)], I),
        "nbody_hermite_create": ([P, C.POINTER(P), I64, C.POINTER(HermiteOpts)], I),
        "nbody_hermite_destroy": ([P], I),
        "nbody_hermite_set_state": ([P, P, Src], I),
        "nbody_hermite_get_state": ([P, P, Src, P, P, P, P, P, P, P, P], I),
        "nbody_hermite_step": ([P, P, C.POINTER(I64), C.POINTER(I64)], I),
        "nbody_hermite_advance": ([P, P, I64, C.POINTER(HermiteStats)], I),
        "nbody_hermite_energy": ([P, P, C.POINTER(D), C.POINTER(D)], I),
        "nbody_hermite_state_bytes": ([P], I64),
        "nbody_hermite_save": ([P, P, P], I),
        "nbody_hermite_load": ([P, P, P], I),
        "nbody_block_level": ([D, I64, I64, I, I], I64),
        "nbody_kernel_timing": ([P, I], I),
        "nbody_force_vjp": ([P, P, I, D, D, I64, Src, P, I64, Src, P, P, P, P, P, P, P, P], I),
        "nbody_force_vjp_self": ([P, P, I, D, D, I64, Src, P, P, P, P, P, P], I),
        "nbody_shared_ckpt_bytes": ([I64, I, I], I64),
        "nbody_force_batched": ([P, P, I, D, C.c_int32, P, P, I64, Src, Out], I),
        "nbody_batch_hermite": ([P, P, I, D, C.c_int32, P, P, I64, D, I, P, P, P, P, P, I], I),
        "nbody_autotune_batched": ([P, P, I, D, C.c_int32, P, P, I64, Src, Out, I, C.POINTER(Tile),
                                    C.POINTER(D)], I),
        "nbody_shared_run": ([P, P, I, D, D, D, I, I64, Src, P, P, P, I], I),
        "nbody_shared_adjoint": ([P, P, I, D, D, D, I, I64, Src, P, I, P, P, P, P, P], I),
        "nbody_kernel_time": ([P, C.POINTER(D), C.POINTER(I64)], I),
        "nbody_force_acc": ([P, P, I, D, D, I64, Src, P, I64, Src, Out], I),
        "nbody_force_nn": ([P, P, I, D, D, I64, Src, P, I64, Src, Out, P, P], I),
        "nbody_leapfrog": ([P, P, I, D, D, D, I, I64, P, P, P, P, P, I], I),
        "GPU_open": ([I], I),
        "GPU_close": ([I], I),
        "GPU_npipes": ([], I),
        "GPU_set_j_particle": ([I, I, I, D, D, P, P, P, P], I),
        "GPU_set_ti": ([I, D], I),
        "GPUcalc_firsthalf": ([I, I, I, P, P, P, D], I),
        "GPUcalc_lasthalf": ([I, I, P, P, P], I),
        "GPUcalc_lasthalf2": ([I, I, P, P, P, P], I),
        "GPU_set_nn": ([I, I], I),
        "GPU_set_precision": ([I, I], I),
        "GPU_last_error": ([I], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def block_level(crit: float, dt_old: int, t_new: int, lmin: int = -20, lmax: int = -3) -> int:
    """The corrector's power-of-two step rule, evaluated on the host."""
    return int(lib().nbody_block_level(float(crit), int(dt_old), int(t_new), int(lmin), int(lmax)))


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _rows(t, n, name, dtype=None):
    """Three row pointers of a (3, n) tensor."""
    torch = _torch()
    dtype = dtype or torch.float64
    if t.dtype != dtype or t.dim() != 2 or t.shape[0] != 3 or t.shape[1] != n:
        raise ValueError(f"{name}: expected a (3, {n}) {dtype} tensor, got {tuple(t.shape)} {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor")
    b = t.data_ptr()
    return [b, b + 8 * n, b + 16 * n]


def _vec(t, n, name, dtype=None):
    torch = _torch()
    dtype = dtype or torch.float64
    if t.dtype != dtype or t.dim() != 1 or t.shape[0] != n or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous ({n},) {dtype} tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor")
    return t.data_ptr()


def _src(x, v, m, n, name):
    xs = _rows(x, n, name + ".x")
    vs = _rows(v, n, name + ".v")
    mp = _vec(m, n, name + ".m") if m is not None else None
    return Src(xs[0], xs[1], xs[2], vs[0], vs[1], vs[2], mp)


class Context:
    """A library context on one GPU (``device=-1``: argument checks only)."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        L = lib()
        h = C.c_void_p()
        rc = L.nbody_create(C.byref(h), int(device),
                            tune_cache.encode() if tune_cache else None)
        if rc != 0:
            raise NBodyError(rc, f"nbody_create(device={device}) failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().nbody_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().nbody_last_error(self._h)
            raise NBodyError(rc, f"{what}: {msg.decode() if msg else ''}")

    def last_error(self) -> str:
        m = lib().nbody_last_error(self._h)
        return m.decode() if m else ""

    def sync(self, stream=None):
        self._check(lib().nbody_sync(self._h, _stream(stream)), "nbody_sync")

    def kernel_timing(self, enable: bool):
        """Start (or stop) timing every pairwise-kernel launch with HIP events."""
        self._check(lib().nbody_kernel_timing(self._h, 1 if enable else 0), "nbody_kernel_timing")

    def kernel_time(self):
        """(total kernel milliseconds, launches) since timing was enabled or
        last read; waits for the recorded events."""
        ms, n = C.c_double(), C.c_int64()
        self._check(lib().nbody_kernel_time(self._h, C.byref(ms), C.byref(n)), "nbody_kernel_time")
        return ms.value, n.value

    def reserve(self, max_i, max_j):
        self._check(lib().nbody_reserve(self._h, int(max_i), int(max_j)), "nbody_reserve")

    def set_tile(self, prec="ds", tile_j=None, ipt=None, wg=None, split=0, jsrc=0, unroll=0, waves=0):
        p = PREC[prec]
        if tile_j is None:
            self._check(lib().nbody_set_tile(self._h, p, None), "nbody_set_tile")
        else:
            t = Tile(int(tile_j), int(ipt), int(wg), int(split), int(jsrc), int(unroll), int(waves))
            self._check(lib().nbody_set_tile(self._h, p, C.byref(t)), "nbody_set_tile")

    def get_tile(self, n_i, n_j, prec="ds"):
        t = Tile()
        self._check(lib().nbody_get_tile(self._h, PREC[prec], int(n_i), int(n_j), C.byref(t)),
                    "nbody_get_tile")
        return t.as_dict()

    def force(self, xi, vi, xj, vj, mj, eps, G=1.0, prec="ds", i_self=None, out=None,
              stream=None, noalloc=False):
        """(acc (3, n_i), jerk (3, n_i), pot (n_i,)) of i due to j; see
        nbody_force.  ``i_self`` is an int32 tensor (n_i,) or None.
        ``noalloc``: call nbody_force_noalloc instead (no device allocation
        inside the library; pass ``out`` to allocate nothing at all)."""
        torch = _torch()
        ni, nj = xi.shape[1], xj.shape[1]
        I = _src(xi, vi, None, ni, "I")
        J = _src(xj, vj, mj, nj, "J")
        if out is None:
            acc = torch.empty((3, ni), dtype=torch.float64, device=xi.device)
            jerk = torch.empty((3, ni), dtype=torch.float64, device=xi.device)
            pot = torch.empty((ni,), dtype=torch.float64, device=xi.device)
        else:
            acc, jerk, pot = out
        a, j = _rows(acc, ni, "acc"), _rows(jerk, ni, "jerk")
        O = Out(a[0], a[1], a[2], j[0], j[1], j[2], _vec(pot, ni, "pot"))
        sp = _vec(i_self, ni, "i_self", torch.int32) if i_self is not None else None
        fn, name = ((lib().nbody_force_noalloc, "nbody_force_noalloc") if noalloc
                    else (lib().nbody_force, "nbody_force"))
        self._check(fn(self._h, _stream(stream), PREC[prec], float(G), float(eps), ni, I, sp, nj, J, O),
                    name)
        return acc, jerk, pot

    def force_acc(self, xi, xj, mj, eps, G=1.0, prec="ds", i_self=None, stream=None):
        """(acc (3, n_i), pot (n_i,)): the force-only evaluation, see
        nbody_force_acc.  No velocities are needed."""
        torch = _torch()
        ni, nj = xi.shape[1], xj.shape[1]
        xs, xjs = _rows(xi, ni, "I.x"), _rows(xj, nj, "J.x")
        I = Src(xs[0], xs[1], xs[2], None, None, None, None)
        J = Src(xjs[0], xjs[1], xjs[2], None, None, None, _vec(mj, nj, "J.m"))
        acc = torch.empty((3, ni), dtype=torch.float64, device=xi.device)
        pot = torch.empty((ni,), dtype=torch.float64, device=xi.device)
        a = _rows(acc, ni, "acc")
        O = Out(a[0], a[1], a[2], None, None, None, _vec(pot, ni, "pot"))
        sp = _vec(i_self, ni, "i_self", torch.int32) if i_self is not None else None
        self._check(lib().nbody_force_acc(self._h, _stream(stream), PREC[prec], float(G), float(eps),
                                          ni, I, sp, nj, J, O), "nbody_force_acc")
        return acc, pot

    def force_nn(self, xi, vi, xj, vj, mj, eps, G=1.0, prec="ds", i_self=None, want_r2=True,
                 stream=None):
        """(acc, jerk, pot, nn (n_i,) int32, nn_r2 (n_i,) or None): nbody_force
        plus the nearest neighbour of each i, see nbody_force_nn."""
        torch = _torch()
        ni, nj = xi.shape[1], xj.shape[1]
        I = _src(xi, vi, None, ni, "I")
        J = _src(xj, vj, mj, nj, "J")
        dev = xi.device
        acc = torch.empty((3, ni), dtype=torch.float64, device=dev)
        jerk = torch.empty((3, ni), dtype=torch.float64, device=dev)
        pot = torch.empty((ni,), dtype=torch.float64, device=dev)
        nn = torch.empty((ni,), dtype=torch.int32, device=dev)
        r2 = torch.empty((ni,), dtype=torch.float64, device=dev) if want_r2 else None
        a, j = _rows(acc, ni, "acc"), _rows(jerk, ni, "jerk")
        O = Out(a[0], a[1], a[2], j[0], j[1], j[2], _vec(pot, ni, "pot"))
        sp = _vec(i_self, ni, "i_self", torch.int32) if i_self is not None else None
        self._check(lib().nbody_force_nn(self._h, _stream(stream), PREC[prec], float(G), float(eps),
                                         ni, I, sp, nj, J, O, nn.data_ptr() if ni else None,
                                         r2.data_ptr() if r2 is not None and ni else None),
                    "nbody_force_nn")
        return acc, jerk, pot, nn, r2

    def leapfrog(self, x, v, m, eps, dt, nsteps, acc=None, G=1.0, prec="ds", want_pot=True,
                 stream=None):
        """Kick-drift-kick run in place on x, v ((3, n) float64); ``acc`` is
        a(x) if known (it is updated in place), else computed first.
        Returns (acc, pot or None) at the end; see nbody_leapfrog."""
        torch = _torch()
        n = x.shape[1]
        _rows(x, n, "x"); _rows(v, n, "v"); _vec(m, n, "m")
        have = acc is not None
        if not have:
            acc = torch.empty((3, n), dtype=torch.float64, device=x.device)
        _rows(acc, n, "acc")
        pot = torch.empty((n,), dtype=torch.float64, device=x.device) if want_pot else None
        ptr = lambda t: t.data_ptr() if t is not None and n else None
        self._check(lib().nbody_leapfrog(self._h, _stream(stream), PREC[prec], float(G), float(eps),
                                         float(dt), int(nsteps), n, ptr(x), ptr(v), ptr(m), ptr(acc),
                                         ptr(pot), 1 if have else 0), "nbody_leapfrog")
        return acc, pot

    def force_vjp(self, xi, vi, xj, vj, mj, eps, ga, gj=None, gp=None, G=1.0, prec="ds",
                  i_self=None, want=("xi", "vi", "xj", "vj", "mj"), stream=None):
        """Cotangents of x_i, v_i, x_j, v_j, m_j for output cotangents (ga, gj,
        gp) of nbody_force; returns a dict with the requested keys."""
        torch = _torch()
        ni, nj = xi.shape[1], xj.shape[1]
        I = _src(xi, vi, None, ni, "I")
        J = _src(xj, vj, mj, nj, "J")
        _rows(ga, ni, "ga")
        if gj is not None:
            _rows(gj, ni, "gj")
        if gp is not None:
            _vec(gp, ni, "gp")
        dev = xi.device
        out = {}
        shapes = {"xi": (3, ni), "vi": (3, ni), "xj": (3, nj), "vj": (3, nj), "mj": (nj,)}
        for k in want:
            out[k] = torch.empty(shapes[k], dtype=torch.float64, device=dev)
        ptr = lambda k: out[k].data_ptr() if k in out and out[k].numel() else None
        sp = _vec(i_self, ni, "i_self", torch.int32) if i_self is not None else None
        self._check(lib().nbody_force_vjp(
            self._h, _stream(stream), PREC[prec], float(G), float(eps), ni, I, sp, nj, J,
            ga.data_ptr() if ni else None, gj.data_ptr() if gj is not None and ni else None,
            gp.data_ptr() if gp is not None and ni else None,
            ptr("xi"), ptr("vi"), ptr("xj"), ptr("vj"), ptr("mj")), "nbody_force_vjp")
        return out

    def force_vjp_self(self, x, v, m, eps, ga, gj=None, gp=None, G=1.0, prec="ds", stream=None):
        """(gx, gv, gm): total cotangents of one self-gravitating set (fused pass)."""
        torch = _torch()
        n = x.shape[1]
        P = _src(x, v, m, n, "P")
        _rows(ga, n, "ga")
        if gj is not None:
            _rows(gj, n, "gj")
        if gp is not None:
            _vec(gp, n, "gp")
        gx = torch.empty((3, n), dtype=torch.float64, device=x.device)
        gv = torch.empty((3, n), dtype=torch.float64, device=x.device)
        gm = torch.empty((n,), dtype=torch.float64, device=x.device)
        self._check(lib().nbody_force_vjp_self(
            self._h, _stream(stream), PREC[prec], float(G), float(eps), n, P,
            ga.data_ptr() if n else None, gj.data_ptr() if gj is not None and n else None,
            gp.data_ptr() if gp is not None and n else None,
            gx.data_ptr() if n else None, gv.data_ptr() if n else None,
            gm.data_ptr() if n else None), "nbody_force_vjp_self")
        return gx, gv, gm

    def shared_run(self, x0, v0, m, eps, dt, nsteps, G=1.0, prec="ds", ckpt_every=8,
                   checkpoints=True, stream=None):
        """Shared-step Hermite run; returns (x_T, v_T, ckpt or None)."""
        torch = _torch()
        n = x0.shape[1]
        P = _src(x0, v0, m, n, "P0")
        xo = torch.empty((3, n), dtype=torch.float64, device=x0.device)
        vo = torch.empty((3, n), dtype=torch.float64, device=x0.device)
        ck = None
        if checkpoints:
            nbytes = lib().nbody_shared_ckpt_bytes(n, int(nsteps), int(ckpt_every))
            ck = torch.empty((nbytes // 8,), dtype=torch.float64, device=x0.device)
        self._check(lib().nbody_shared_run(self._h, _stream(stream), PREC[prec], float(G), float(eps),
                                           float(dt), int(nsteps), n, P, xo.data_ptr(), vo.data_ptr(),
                                           ck.data_ptr() if ck is not None else None, int(ckpt_every)),
                    "nbody_shared_run")
        return xo, vo, ck

    def shared_adjoint(self, x0, v0, m, eps, dt, nsteps, ckpt, gx_end, gv_end=None, G=1.0, prec="ds",
                       ckpt_every=8, stream=None):
        """(gx0, gv0, gm) of L = <gx_end, x_T> + <gv_end, v_T>."""
        torch = _torch()
        n = x0.shape[1]
        P = _src(x0, v0, m, n, "P0")
        _rows(gx_end, n, "gx_end")
        if gv_end is not None:
            _rows(gv_end, n, "gv_end")
        gx = torch.empty((3, n), dtype=torch.float64, device=x0.device)
        gv = torch.empty((3, n), dtype=torch.float64, device=x0.device)
        gm = torch.empty((n,), dtype=torch.float64, device=x0.device)
        self._check(lib().nbody_shared_adjoint(
            self._h, _stream(stream), PREC[prec], float(G), float(eps), float(dt), int(nsteps), n, P,
            ckpt.data_ptr() if ckpt is not None else None, int(ckpt_every), gx_end.data_ptr(),
            gv_end.data_ptr() if gv_end is not None else None, gx.data_ptr(), gv.data_ptr(),
            gm.data_ptr()), "nbody_shared_adjoint")
        return gx, gv, gm

    def force_batched(self, x, v, m, offsets, eps, G=1.0, prec="ds", out=None, stream=None):
        """Forces of independent clusters (concatenated rows); offsets int64
        (C+1,) and eps float64 (C,) are GPU tensors.  Returns (acc, jerk, pot)."""
        torch = _torch()
        n = x.shape[1]
        C_ = int(eps.shape[0])
        P = _src(x, v, m, n, "P")
        if out is None:
            acc = torch.empty((3, n), dtype=torch.float64, device=x.device)
            jerk = torch.empty((3, n), dtype=torch.float64, device=x.device)
            pot = torch.empty((n,), dtype=torch.float64, device=x.device)
        else:
            acc, jerk, pot = out
        a, j = _rows(acc, n, "acc"), _rows(jerk, n, "jerk")
        O = Out(a[0], a[1], a[2], j[0], j[1], j[2], _vec(pot, n, "pot"))
        op = _vec(offsets, C_ + 1, "offsets", torch.int64)
        ep = _vec(eps, C_, "eps") if C_ else None
        self._check(lib().nbody_force_batched(self._h, _stream(stream), PREC[prec], float(G), C_, op, ep,
                                              n, P, O), "nbody_force_batched")
        return acc, jerk, pot

    def batch_hermite(self, x, v, a, j, m, offsets, eps, dt, nsteps, G=1.0, prec="ds", use_graph=True,
                      stream=None):
        """Advance every cluster nsteps shared Hermite steps in place."""
        torch = _torch()
        n = x.shape[1]
        C_ = int(eps.shape[0])
        for t, nm in ((x, "x"), (v, "v"), (a, "a"), (j, "j")):
            _rows(t, n, nm)
        _vec(m, n, "m")
        op = _vec(offsets, C_ + 1, "offsets", torch.int64)
        ep = _vec(eps, C_, "eps") if C_ else None
        self._check(lib().nbody_batch_hermite(self._h, _stream(stream), PREC[prec], float(G), C_, op, ep, n,
                                              float(dt), int(nsteps), x.data_ptr(), v.data_ptr(), a.data_ptr(),
                                              j.data_ptr(), m.data_ptr(), 1 if use_graph else 0),
                    "nbody_batch_hermite")

    def autotune_batched(self, x, v, m, offsets, eps, G=1.0, prec="ds", reps=2, stream=None):
        torch = _torch()
        n = x.shape[1]
        C_ = int(eps.shape[0])
        P = _src(x, v, m, n, "P")
        acc = torch.empty((3, n), dtype=torch.float64, device=x.device)
        jerk = torch.empty((3, n), dtype=torch.float64, device=x.device)
        pot = torch.empty((n,), dtype=torch.float64, device=x.device)
        a, j = _rows(acc, n, "acc"), _rows(jerk, n, "jerk")
        O = Out(a[0], a[1], a[2], j[0], j[1], j[2], _vec(pot, n, "pot"))
        t = Tile()
        ms = C.c_double()
        self._check(lib().nbody_autotune_batched(self._h, _stream(stream), PREC[prec], float(G), C_,
                                                 _vec(offsets, C_ + 1, "offsets", torch.int64),
                                                 _vec(eps, C_, "eps"), n, P, O, int(reps), C.byref(t),
                                                 C.byref(ms)), "nbody_autotune_batched")
        return t.as_dict(), ms.value

    def autotune(self, xi, vi, xj, vj, mj, eps, G=1.0, prec="ds", reps=2, stream=None):
        torch = _torch()
        ni, nj = xi.shape[1], xj.shape[1]
        I = _src(xi, vi, None, ni, "I")
        J = _src(xj, vj, mj, nj, "J")
        acc = torch.empty((3, ni), dtype=torch.float64, device=xi.device)
        jerk = torch.empty((3, ni), dtype=torch.float64, device=xi.device)
        pot = torch.empty((ni,), dtype=torch.float64, device=xi.device)
        a, j = _rows(acc, ni, "acc"), _rows(jerk, ni, "jerk")
        O = Out(a[0], a[1], a[2], j[0], j[1], j[2], _vec(pot, ni, "pot"))
        t = Tile()
        ms = C.c_double()
        self._check(lib().nbody_autotune(self._h, _stream(stream), PREC[prec], float(G),
                                         float(eps), ni, I, nj, J, O, int(reps), C.byref(t),
                                         C.byref(ms)), "nbody_autotune")
        return t.as_dict(), ms.value

    def select_active(self, t, dt, stream=None):
        """(idx int32 tensor (n_act,), t_next) of the next block."""
        torch = _torch()
        n = t.shape[0]
        idx = torch.empty((max(n, 1),), dtype=torch.int32, device=t.device)
        na, tn = C.c_int64(), C.c_int64()
        tp = _vec(t, n, "t", torch.int64) if n else None
        dp = _vec(dt, n, "dt", torch.int64) if n else None
        self._check(lib().nbody_select_active(self._h, _stream(stream), n, tp, dp,
                                              idx.data_ptr(), C.byref(na), C.byref(tn)),
                    "nbody_select_active")
        return idx[:na.value], tn.value

    def hermite(self, n, *, G=1.0, eps=0.0, eta=0.02, eta_start=0.01, dt_min_log2=-20,
                dt_max_log2=-3, shared_dt_log2=0, prec="ds"):
        return Hermite(self, n, HermiteOpts(float(G), float(eps), float(eta), float(eta_start),
                                            int(dt_min_log2), int(dt_max_log2),
                                            int(shared_dt_log2), PREC[prec]))


class Hermite:
    """Device-resident Hermite block-step integrator (nbody_hermite_*)."""

    def __init__(self, ctx: Context, n: int, opts: HermiteOpts):
        self.ctx = ctx
        self.n = int(n)
        self.opts = opts
        h = C.c_void_p()
        ctx._check(lib().nbody_hermite_create(ctx.handle, C.byref(h), self.n, C.byref(opts)),
                   "nbody_hermite_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().nbody_hermite_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, x, v, m, stream=None):
        self.ctx._check(lib().nbody_hermite_set_state(self._h, _stream(stream),
                                                      _src(x, v, m, self.n, "P")),
                        "nbody_hermite_set_state")

    def get_state(self, stream=None):
        """dict of x, v (3, n), m (n,), a, jerk (3, n), t, dt (n,) int64."""
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        n = self.n
        x = torch.empty((3, n), dtype=torch.float64, device=dev)
        v = torch.empty((3, n), dtype=torch.float64, device=dev)
        m = torch.empty((n,), dtype=torch.float64, device=dev)
        a = torch.empty((3, n), dtype=torch.float64, device=dev)
        j = torch.empty((3, n), dtype=torch.float64, device=dev)
        t = torch.empty((n,), dtype=torch.int64, device=dev)
        dt = torch.empty((n,), dtype=torch.int64, device=dev)
        ar, jr = _rows(a, n, "a"), _rows(j, n, "j")
        self.ctx._check(lib().nbody_hermite_get_state(self._h, _stream(stream), _src(x, v, m, n, "P"),
                                                      ar[0], ar[1], ar[2], jr[0], jr[1], jr[2],
                                                      t.data_ptr(), dt.data_ptr()),
                        "nbody_hermite_get_state")
        return {"x": x, "v": v, "m": m, "a": a, "jerk": j, "t": t, "dt": dt}

    def step(self, stream=None):
        na, tt = C.c_int64(), C.c_int64()
        self.ctx._check(lib().nbody_hermite_step(self._h, _stream(stream), C.byref(na), C.byref(tt)),
                        "nbody_hermite_step")
        return na.value, tt.value

    def advance(self, t_end_ticks, stream=None):
        st = HermiteStats()
        self.ctx._check(lib().nbody_hermite_advance(self._h, _stream(stream), int(t_end_ticks),
                                                    C.byref(st)), "nbody_hermite_advance")
        return {"steps": st.steps, "sum_active": st.sum_active, "t_ticks": st.t_ticks}

    def energy(self, stream=None):
        ek, ep = C.c_double(), C.c_double()
        self.ctx._check(lib().nbody_hermite_energy(self._h, _stream(stream), C.byref(ek), C.byref(ep)),
                        "nbody_hermite_energy")
        return ek.value, ep.value

    def save(self, stream=None) -> bytes:
        nbytes = lib().nbody_hermite_state_bytes(self._h)
        buf = C.create_string_buffer(nbytes)
        self.ctx._check(lib().nbody_hermite_save(self._h, _stream(stream), buf), "nbody_hermite_save")
        return buf.raw

    def load(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(blob, len(blob))
        self.ctx._check(lib().nbody_hermite_load(self._h, _stream(stream), buf), "nbody_hermite_load")


class Grape:
    """The GRAPE-6-style calls of include/nbody_grape.h on one cluster, with
    numpy marshalling (host arrays, as the interface takes)."""

    def __init__(self, clusterid: int = 0):
        self.id = int(clusterid)
        self._call("GPU_open", self.id)

    def _call(self, name, *args):
        rc = getattr(lib(), name)(*args)
        if rc != 0:
            raise NBodyError(rc, f"{name}: {lib().GPU_last_error(self.id).decode(errors='replace')}")

    def close(self):
        self._call("GPU_close", self.id)

    def set_j_particle(self, address, index, tj, mass, x, v, a, j):
        import numpy as np
        vec = [np.ascontiguousarray(q, dtype=np.float64) for q in (x, v, a, j)]
        self._call("GPU_set_j_particle", self.id, int(address), int(index), float(tj), float(mass),
                   *[q.ctypes.data_as(C.c_void_p) for q in vec])

    def set_ti(self, ti):
        self._call("GPU_set_ti", self.id, float(ti))

    def set_nn(self, enable):
        self._call("GPU_set_nn", self.id, 1 if enable else 0)

    def set_precision(self, prec):
        self._call("GPU_set_precision", self.id, PREC[prec])

    def calc_firsthalf(self, nj, index, xi, vi, eps2):
        """xi, vi: (ni, 3) arrays; index: (ni,) identities."""
        import numpy as np
        idx = np.ascontiguousarray(index, dtype=np.int32)
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
        vi = np.ascontiguousarray(vi, dtype=np.float64).reshape(-1, 3)
        self._keep = (idx, xi, vi)
        ptr = lambda q: q.ctypes.data_as(C.c_void_p) if q.size else None
        self._call("GPUcalc_firsthalf", self.id, int(nj), idx.size, ptr(idx), ptr(xi), ptr(vi), float(eps2))

    def calc_lasthalf(self, ni, nn=False):
        """Returns (acc (ni, 3), jerk (ni, 3), pot (ni,)) and, with nn, the
        nearest-neighbour identities (ni,)."""
        import numpy as np
        acc = np.empty((ni, 3)); jerk = np.empty((ni, 3)); pot = np.empty(ni)
        ptr = lambda q: q.ctypes.data_as(C.c_void_p) if q.size else None
        if nn:
            nnb = np.empty(ni, dtype=np.int32)
            self._call("GPUcalc_lasthalf2", self.id, int(ni), ptr(acc), ptr(jerk), ptr(pot), ptr(nnb))
            return acc, jerk, pot, nnb
        self._call("GPUcalc_lasthalf", self.id, int(ni), ptr(acc), ptr(jerk), ptr(pot))
        return acc, jerk, pot
