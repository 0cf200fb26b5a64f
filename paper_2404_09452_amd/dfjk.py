"""Python binding of the DF-J/K library (argument marshalling only).

Every step of the build runs in the HIP kernels behind the C ABI; this module
turns numpy/torch arguments into pointers, allocates the device workspaces
with torch and passes torch's current HIP stream.
"""
from __future__ import annotations

import ctypes
import functools

import numpy as np
import torch

from . import _native as N

FP64, MIXED_FP32, MIXED_BF16X3, MIXED_INT8, MIXED_INT8_FAST = 0, 1, 2, 3, 4
PRECISION = {"fp64": FP64, "fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3, "int8": MIXED_INT8,
             "int8_fast": MIXED_INT8_FAST}
EXPORT_INT3C, EXPORT_B, EXPORT_METRIC, EXPORT_CHOL = 0, 1, 2, 3

STATUS = {0: "OK", 1: "INVALID", 2: "UNSUPPORTED", 3: "NOT_POSDEF", 4: "OOM", 5: "DEVICE",
          6: "NO_DEVICE", 7: "STATE"}


class DFJKError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("dfjk %s: %s" % (STATUS.get(code, code), message))
        self.code = code
        self.status = STATUS.get(code, str(code))
        self.message = message


def _check(rc):
    if rc != 0:
        msg = N.lib().dfjk_last_error()
        raise DFJKError(rc, msg.decode() if msg else "")


def _on_stream(fn):
    """Run a call's own device work (input copies, output and scratch
    allocations) on the stream the library is given, so that the library
    never reads an input before its copy, nor memory that the caching
    allocator has already handed to work on another stream."""
    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kw):
        if stream is None:
            return fn(*args, stream=None, **kw)
        with torch.cuda.stream(stream):
            return fn(*args, stream=stream, **kw)
    return wrapper


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """One molecule: host preparation at construction, then screen/setup once
    and build any number of times.

    coords: (natm, 3) Bohr; ao and aux: (atom, l, exponent) arrays."""

    def __init__(self, coords, ao_atom, ao_l, ao_exp, aux_atom, aux_l, aux_exp, schwarz_thresh=1e-14,
                 aux_slab=0, k_tile=0):
        L = N.lib()
        self._keep = []
        coords = np.ascontiguousarray(coords, dtype=np.float64)

        def basis(atom, l, e):
            a = np.ascontiguousarray(atom, dtype=np.int32)
            ll = np.ascontiguousarray(l, dtype=np.int32)
            ee = np.ascontiguousarray(e, dtype=np.float64)
            self._keep += [a, ll, ee]
            return N.Basis(len(ll), a.ctypes.data_as(N.P_i32), ll.ctypes.data_as(N.P_i32),
                           ee.ctypes.data_as(N.P_dbl))

        ao = basis(ao_atom, ao_l, ao_exp)
        aux = basis(aux_atom, aux_l, aux_exp)
        opt = N.Options(float(schwarz_thresh), int(aux_slab), int(k_tile))
        h = ctypes.c_void_p()
        _check(L.dfjk_plan_create(len(coords), coords.ctypes.data_as(N.P_dbl), ctypes.byref(ao),
                                  ctypes.byref(aux), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self._ws = None
        self._scratch = {}
        self._dscratch = {}
        inf = self.info()
        self.nao, self.naux = inf["nao"], inf["naux"]

    @classmethod
    def from_molecule(cls, mol, schwarz_thresh=1e-14, aux_slab=0, k_tile=0):
        return cls(mol.coords, mol.ao_atom, mol.ao_l, mol.ao_exp, mol.aux_atom, mol.aux_l, mol.aux_exp,
                   schwarz_thresh=schwarz_thresh, aux_slab=aux_slab, k_tile=k_tile)

    # -- facts -------------------------------------------------------------
    def info(self):
        inf = N.Info()
        _check(N.lib().dfjk_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in N.Info._fields_}

    def aux_order(self):
        out = np.zeros(self.naux, dtype=np.int32)
        _check(N.lib().dfjk_plan_aux_order(self._h, out.ctypes.data_as(N.P_i32)))
        return out

    # -- phases ------------------------------------------------------------
    @_on_stream
    def screen(self, stream=None):
        n = ctypes.c_size_t()
        _check(N.lib().dfjk_screen_bytes(self._h, ctypes.byref(n)))
        scratch = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
        _check(N.lib().dfjk_screen(self._h, _ptr(scratch), n.value, _stream_handle(stream)))
        return self

    def setup_bytes(self):
        n = ctypes.c_size_t()
        _check(N.lib().dfjk_setup_bytes(self._h, ctypes.byref(n)))
        return n.value

    @_on_stream
    def setup(self, stream=None):
        nbytes = self.setup_bytes()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(N.lib().dfjk_setup(self._h, _ptr(self._ws), self._ws.numel(), _stream_handle(stream)))
        return self

    @_on_stream
    def setup_host(self, max_device_bytes=0, stream=None):
        """Set up with B formed block by block straight into page-locked host
        memory (dfjk_setup_host): the device workspace stays within
        max_device_bytes (0: no limit).  Returns self; self.setup_host_info
        holds the host and device byte counts."""
        hb, db = ctypes.c_size_t(), ctypes.c_size_t()
        _check(N.lib().dfjk_setup_host_bytes(self._h, int(max_device_bytes), ctypes.byref(hb), ctypes.byref(db)))
        self._host_B = torch.empty(hb.value, dtype=torch.uint8, pin_memory=True)
        self._ws = torch.empty(db.value, dtype=torch.uint8, device="cuda")
        _check(N.lib().dfjk_setup_host(self._h, ctypes.c_void_p(self._host_B.data_ptr()), hb.value, _ptr(self._ws),
                                       self._ws.numel(), _stream_handle(stream)))
        self._scratch = {}
        self.setup_host_info = {"host_bytes": hb.value, "device_bytes": db.value}
        return self

    def build_bytes(self, nocc, precision="fp64", with_density=False):
        n = ctypes.c_size_t()
        _check(N.lib().dfjk_build_bytes(self._h, int(nocc), PRECISION[precision], int(with_density),
                                        ctypes.byref(n)))
        return n.value

    def scratch(self, nocc, precision="fp64", with_density=False):
        key = (int(nocc), precision, bool(with_density))
        if key not in self._scratch:
            self._scratch[key] = torch.empty(self.build_bytes(nocc, precision, with_density),
                                             dtype=torch.uint8, device="cuda")
        return self._scratch[key]

    @_on_stream
    def build(self, C=None, D=None, precision="fp64", out=None, stream=None):
        """J, K (nao x nao) and E = [E_J, E_K] as float64 CUDA tensors."""
        if (C is None) == (D is None):
            raise ValueError("give exactly one of C and D")
        dev = torch.device("cuda")
        if C is not None:
            C = torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous()
            if C.dim() != 2 or C.shape[0] != self.nao:
                raise ValueError("C must be (nao, nocc)")
            nocc = C.shape[1]
        else:
            D = torch.as_tensor(D, dtype=torch.float64, device=dev).contiguous()
            if tuple(D.shape) != (self.nao, self.nao):
                raise ValueError("D must be (nao, nao)")
            nocc = 0
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        scr = self.scratch(nocc if C is not None else 1, precision, D is not None)
        _check(N.lib().dfjk_build(self._h, _ptr(C), int(nocc), _ptr(D), PRECISION[precision], _ptr(J),
                                  _ptr(K), _ptr(E), _ptr(scr), scr.numel(), _stream_handle(stream)))
        return J, K, E

    @_on_stream
    def build_checked(self, C, budget=1e-6, out=None, stream=None):
        """The precision chosen against an energy-error budget (Eh) through
        dfjk_build_checked: int8 when its rigorous bound is within the
        budget, else FP64.  Returns (J, K, E, chosen, bound) with chosen
        "int8" or "fp64"."""
        dev = torch.device("cuda")
        C = torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous()
        if C.dim() != 2 or C.shape[0] != self.nao:
            raise ValueError("C must be (nao, nocc)")
        nocc = C.shape[1]
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        key = (int(nocc), "checked", False)
        if key not in self._scratch:
            n = ctypes.c_size_t()
            _check(N.lib().dfjk_build_checked_bytes(self._h, int(nocc), ctypes.byref(n)))
            self._scratch[key] = torch.empty(n.value, dtype=torch.uint8, device=dev)
        scr = self._scratch[key]
        chosen, bound = ctypes.c_int32(), ctypes.c_double()
        _check(N.lib().dfjk_build_checked(self._h, _ptr(C), int(nocc), float(budget), _ptr(J), _ptr(K), _ptr(E),
                                          _ptr(scr), scr.numel(), _stream_handle(stream), ctypes.byref(chosen),
                                          ctypes.byref(bound)))
        name = {v: k for k, v in PRECISION.items()}[chosen.value]
        return J, K, E, name, bound.value

    @_on_stream
    def build_static(self, C=None, D=None, precision="fp64", out=None, stream=None):
        """As build, through dfjk_build_static: the library's static device
        scratch instead of a workspace, so the call allocates nothing in the
        library (outputs are allocated here unless `out` is given)."""
        if (C is None) == (D is None):
            raise ValueError("give exactly one of C and D")
        dev = torch.device("cuda")
        if C is not None:
            C = torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous()
            if C.dim() != 2 or C.shape[0] != self.nao:
                raise ValueError("C must be (nao, nocc)")
            nocc = C.shape[1]
        else:
            D = torch.as_tensor(D, dtype=torch.float64, device=dev).contiguous()
            if tuple(D.shape) != (self.nao, self.nao):
                raise ValueError("D must be (nao, nao)")
            nocc = 0
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        _check(N.lib().dfjk_build_static(self._h, _ptr(C), int(nocc), _ptr(D), PRECISION[precision], _ptr(J),
                                         _ptr(K), _ptr(E), _stream_handle(stream)))
        return J, K, E

    def build_delta_bytes(self, nocc, precision="fp32"):
        n = ctypes.c_size_t()
        _check(N.lib().dfjk_build_delta_bytes(self._h, int(nocc), PRECISION[precision], ctypes.byref(n)))
        return n.value

    @_on_stream
    def build_delta(self, C, C0, K0, precision="fp32", out=None, stream=None):
        """K = K0 + K(D - D0) with the correction in `precision`; J, E in FP64.
        K0 must be the FP64 K of C0 from build() on this plan."""
        dev = torch.device("cuda")
        C = torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous()
        C0 = torch.as_tensor(C0, dtype=torch.float64, device=dev).contiguous()
        K0 = torch.as_tensor(K0, dtype=torch.float64, device=dev).contiguous()
        if C.shape != C0.shape or C.dim() != 2 or C.shape[0] != self.nao:
            raise ValueError("C and C0 must both be (nao, nocc)")
        if tuple(K0.shape) != (self.nao, self.nao):
            raise ValueError("K0 must be (nao, nao)")
        nocc = C.shape[1]
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        key = ("delta", int(nocc), precision)
        if key not in self._scratch:
            self._scratch[key] = torch.empty(self.build_delta_bytes(nocc, precision), dtype=torch.uint8,
                                             device=dev)
        scr = self._scratch[key]
        _check(N.lib().dfjk_build_delta(self._h, _ptr(C), _ptr(C0), int(nocc), _ptr(K0), PRECISION[precision],
                                        _ptr(J), _ptr(K), _ptr(E), _ptr(scr), scr.numel(), _stream_handle(stream)))
        return J, K, E

    @_on_stream
    def build_uks(self, Ca, Cb, precision="fp64", out=None, stream=None):
        """Open-shell build: J (from D_a + D_b), K_a, K_b and E = [E_J, E_K] with
        D_s = C_s C_s^T; Cb (or Ca) may have zero columns."""
        dev = torch.device("cuda")
        Cs = []
        for C in (Ca, Cb):
            C = torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous()
            if C.dim() != 2 or C.shape[0] != self.nao:
                raise ValueError("C_a and C_b must be (nao, nocc_s)")
            Cs.append(C)
        na, nb = Cs[0].shape[1], Cs[1].shape[1]
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            Ka, Kb = torch.empty_like(J), torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, Ka, Kb, E = out
        key = ("uks", int(na), int(nb), precision)
        if key not in self._scratch:
            n = ctypes.c_size_t()
            _check(N.lib().dfjk_build_uks_bytes(self._h, int(na), int(nb), PRECISION[precision], ctypes.byref(n)))
            self._scratch[key] = torch.empty(n.value, dtype=torch.uint8, device=dev)
        scr = self._scratch[key]
        _check(N.lib().dfjk_build_uks(self._h, _ptr(Cs[0]) if na else ctypes.c_void_p(0), int(na),
                                      _ptr(Cs[1]) if nb else ctypes.c_void_p(0), int(nb), PRECISION[precision],
                                      _ptr(J), _ptr(Ka), _ptr(Kb), _ptr(E), _ptr(scr), scr.numel(),
                                      _stream_handle(stream)))
        return J, Ka, Kb, E

    def build_shape(self, nocc, precision="fp64"):
        """The K launch shape of a C-route build (dfjk_build_shape):
        {"k_tile", "nsplit", "aux_slab", "nslab"}."""
        out = (ctypes.c_int32 * 4)()
        _check(N.lib().dfjk_build_shape(self._h, int(nocc), PRECISION[precision], out))
        return dict(zip(("k_tile", "nsplit", "aux_slab", "nslab"), (int(v) for v in out)))

    @_on_stream
    def autotune(self, C, precision="fp64", stream=None):
        """Time the candidate tile shapes and split counts of the K contraction
        for this C shape (dfjk_autotune) and keep the fastest; returns
        ((tile, split), {(tile, split): ms})."""
        C = torch.as_tensor(C, dtype=torch.float64, device="cuda").contiguous()
        nocc = C.shape[1]
        nb = ctypes.c_size_t()
        _check(N.lib().dfjk_autotune_bytes(self._h, int(nocc), PRECISION[precision], ctypes.byref(nb)))
        scr = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        chosen, ncand = ctypes.c_int32(), ctypes.c_int32(16)
        cand = (ctypes.c_int32 * 16)()
        ms = (ctypes.c_double * 16)()
        _check(N.lib().dfjk_autotune(self._h, _ptr(C), int(nocc), PRECISION[precision], _ptr(scr), scr.numel(),
                                     _stream_handle(stream), ctypes.byref(chosen), ctypes.byref(ncand), cand, ms))
        self._scratch = {}          # build sizes may have changed
        dec = lambda c: (int(c) // 1000, int(c) % 1000)   # noqa: E731  (1000 * tile + split)
        return dec(chosen.value), {dec(cand[i]): float(ms[i]) for i in range(ncand.value)}

    @_on_stream
    def offload(self, stream=None):
        """Move B to page-locked host memory (dfjk_offload); later builds stream
        it back slab by slab.  Frees the device setup workspace."""
        hb, db = ctypes.c_size_t(), ctypes.c_size_t()
        _check(N.lib().dfjk_offload_bytes(self._h, ctypes.byref(hb), ctypes.byref(db)))
        self._host_B = torch.empty(hb.value, dtype=torch.uint8, pin_memory=True)
        self._tables = torch.empty(max(db.value, 1), dtype=torch.uint8, device="cuda")
        _check(N.lib().dfjk_offload(self._h, ctypes.c_void_p(self._host_B.data_ptr()), hb.value,
                                    _ptr(self._tables), self._tables.numel(), _stream_handle(stream)))
        self._ws = None
        self._scratch = {}
        return self

    # -- diagnostics -------------------------------------------------------
    NSTAGES = 12

    def profile(self, on=True):
        """Record HIP events around every stage of later setups and builds."""
        _check(N.lib().dfjk_profile(self._h, int(bool(on))))
        return self

    def profile_read(self):
        """{stage name: (summed ms, launches)} since the last read; waits for the events."""
        ms = np.zeros(self.NSTAGES)
        cnt = np.zeros(self.NSTAGES, dtype=np.int32)
        _check(N.lib().dfjk_profile_read(self._h, ms.ctypes.data_as(N.P_dbl), cnt.ctypes.data_as(N.P_i32)))
        return {N.lib().dfjk_stage_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(self.NSTAGES)}

    @_on_stream
    def export(self, kind, stream=None):
        if kind in (EXPORT_INT3C, EXPORT_B):
            shape = (self.naux, self.nao, self.nao)
        else:
            shape = (self.naux, self.naux)
        out = torch.empty(shape, dtype=torch.float64, device="cuda")
        _check(N.lib().dfjk_export(self._h, int(kind), _ptr(out), _stream_handle(stream)))
        return out

    @_on_stream
    def sample(self, kind, idx, stream=None):
        idx = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device="cuda").contiguous()
        n = idx.shape[0]
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(N.lib().dfjk_sample(self._h, int(kind), n, _ptr(idx), _ptr(out), _stream_handle(stream)))
        return out

    # -- four-centre direct J/K ---------------------------------------------
    @_on_stream
    def direct_setup(self, stream=None):
        """Pair tables of the four-centre direct path (needs screen(), not setup())."""
        n = ctypes.c_size_t()
        _check(N.lib().dfjk_direct_bytes(self._h, ctypes.byref(n)))
        self._dtables = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
        _check(N.lib().dfjk_direct_setup(self._h, _ptr(self._dtables), self._dtables.numel(), _stream_handle(stream)))
        self._dscratch = {}
        return self

    def direct_stats(self):
        """Kept shell pairs per class (ss, ps, pp, ds, dp, dd) and the screened
        (bra pair, ket pair) combinations."""
        pairs = (ctypes.c_int64 * 6)()
        q = ctypes.c_int64()
        _check(N.lib().dfjk_direct_stats(self._h, pairs, ctypes.byref(q)))
        return {"pairs": [int(x) for x in pairs], "quartets": int(q.value)}

    @_on_stream
    def direct_build(self, C=None, D=None, out=None, stream=None):
        """Exact J, K and E = [E_J, E_K] from four-centre integrals (FP64);
        give exactly one of C (nao x nocc, D = 2 C C^T) and D (symmetric)."""
        if (C is None) == (D is None):
            raise ValueError("give exactly one of C and D")
        dev = torch.device("cuda")
        withD = D is not None
        X = torch.as_tensor(D if withD else C, dtype=torch.float64, device=dev).contiguous()
        if withD and tuple(X.shape) != (self.nao, self.nao):
            raise ValueError("D must be (nao, nao)")
        if not withD and (X.dim() != 2 or X.shape[0] != self.nao):
            raise ValueError("C must be (nao, nocc)")
        nocc = 0 if withD else X.shape[1]
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        if withD not in self._dscratch:
            n = ctypes.c_size_t()
            _check(N.lib().dfjk_direct_build_bytes(self._h, int(withD), ctypes.byref(n)))
            self._dscratch[withD] = torch.empty(n.value, dtype=torch.uint8, device=dev)
        scr = self._dscratch[withD]
        _check(N.lib().dfjk_direct_build(self._h, ctypes.c_void_p(0) if withD else _ptr(X), int(nocc),
                                         _ptr(X) if withD else ctypes.c_void_p(0), _ptr(J), _ptr(K), _ptr(E),
                                         _ptr(scr), scr.numel(), _stream_handle(stream)))
        return J, K, E

    @_on_stream
    def direct_build_delta(self, D, D0, J0, K0, out=None, stream=None):
        """Incremental exact J, K = J0, K0 + J, K(D - D0) with the
        density-weighted Schwarz screen; E from the full D."""
        dev = torch.device("cuda")
        ins = [torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous() for x in (D, D0, J0, K0)]
        for x in ins:
            if tuple(x.shape) != (self.nao, self.nao):
                raise ValueError("D, D0, J0 and K0 must be (nao, nao)")
        if out is None:
            J = torch.empty((self.nao, self.nao), dtype=torch.float64, device=dev)
            K = torch.empty_like(J)
            E = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            J, K, E = out
        if "delta" not in self._dscratch:
            n = ctypes.c_size_t()
            _check(N.lib().dfjk_direct_build_delta_bytes(self._h, ctypes.byref(n)))
            self._dscratch["delta"] = torch.empty(n.value, dtype=torch.uint8, device=dev)
        scr = self._dscratch["delta"]
        _check(N.lib().dfjk_direct_build_delta(self._h, *(_ptr(x) for x in ins), _ptr(J), _ptr(K), _ptr(E),
                                               _ptr(scr), scr.numel(), _stream_handle(stream)))
        return J, K, E

    def close(self):
        if getattr(self, "_h", None):
            N.lib().dfjk_plan_destroy(self._h)
            self._h = None
        self._ws = None
        self._scratch = {}
        self._host_B = None
        self._tables = None
        self._dtables = None
        self._dscratch = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@_on_stream
def setup_batch(plans, stream=None):
    """dfjk_setup_batch: set up several screened plans in one call, the
    integrals of all of them in shared launches per class and each plan's
    factor chain beside the others'.  Each plan keeps its workspace as after
    Plan.setup.  Returns the list of plans."""
    plans = list(plans)
    n = len(plans)
    if n == 0:
        return plans
    for p in plans:
        nbytes = p.setup_bytes()
        if p._ws is None or p._ws.numel() < nbytes:
            p._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    w = (ctypes.c_void_p * n)(*[p._ws.data_ptr() for p in plans])
    b = (ctypes.c_size_t * n)(*[p._ws.numel() for p in plans])
    _check(N.lib().dfjk_setup_batch(n, h, w, b, _stream_handle(stream)))
    return plans


class Batch:
    """Closed-shell builds of several set-up plans in one dfjk_build_batch call:
    grouped K, reduction and energy launches across the molecules.  The scratch
    is kept for the same (plans, nocc, precision)."""

    @staticmethod
    def bytes_needed(plans, noccs, precision="fp64"):
        n = len(plans)
        h = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        k = (ctypes.c_int32 * n)(*[int(x) for x in noccs])
        nb = ctypes.c_size_t()
        _check(N.lib().dfjk_build_batch_bytes(n, h, k, PRECISION[precision], ctypes.byref(nb)))
        return nb.value

    def __init__(self, plans, noccs, precision="fp64", scratch=None):
        """scratch: an optional uint8 CUDA tensor to use when it is large enough."""
        self.plans = list(plans)
        self.noccs = [int(n) for n in noccs]
        self.precision = precision
        n = len(self.plans)
        self._h = (ctypes.c_void_p * n)(*[p._h.value for p in self.plans])
        self._nocc = (ctypes.c_int32 * n)(*self.noccs)
        self.bytes = self.bytes_needed(self.plans, self.noccs, precision)
        nb = ctypes.c_size_t(self.bytes)
        if scratch is not None and scratch.numel() >= nb.value:
            self.scratch = scratch
        else:
            self.scratch = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")

    @_on_stream
    def build(self, Cs, outs=None, stream=None):
        """Cs: list of (nao_i, nocc_i) orbitals; returns [(J, K, E), ...]."""
        dev = torch.device("cuda")
        n = len(self.plans)
        if len(Cs) != n:
            raise ValueError("one C per plan")
        Cs = [torch.as_tensor(C, dtype=torch.float64, device=dev).contiguous() for C in Cs]
        for C, p, k in zip(Cs, self.plans, self.noccs):
            if tuple(C.shape) != (p.nao, k):
                raise ValueError("C must be (nao, nocc) of its plan")
        if outs is None:
            outs = []
            for p in self.plans:
                J = torch.empty((p.nao, p.nao), dtype=torch.float64, device=dev)
                outs.append((J, torch.empty_like(J), torch.empty(2, dtype=torch.float64, device=dev)))
        arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])   # noqa: E731
        _check(N.lib().dfjk_build_batch(n, self._h, arr(Cs), self._nocc, PRECISION[self.precision],
                                        arr([o[0] for o in outs]), arr([o[1] for o in outs]),
                                        arr([o[2] for o in outs]), _ptr(self.scratch), self.scratch.numel(),
                                        _stream_handle(stream)))
        return outs


def build_host(coords, ao_atom, ao_l, ao_exp, aux_atom, aux_l, aux_exp, C=None, D=None, precision="fp64",
               schwarz_thresh=1e-14):
    """One synchronous build from host arrays (dfjk_build_host): returns numpy
    J, K and E = [E_J, E_K].  The library allocates its own device memory for
    the call; use Plan for repeated builds."""
    if (C is None) == (D is None):
        raise ValueError("give exactly one of C and D")
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    def basis(atom, l, e):
        a, ll, ee = arr(atom, np.int32), arr(l, np.int32), arr(e, np.float64)
        return N.Basis(len(ll), a.ctypes.data_as(N.P_i32), ll.ctypes.data_as(N.P_i32), ee.ctypes.data_as(N.P_dbl))

    xyz = arr(coords, np.float64)
    ao, aux = basis(ao_atom, ao_l, ao_exp), basis(aux_atom, aux_l, aux_exp)
    nao = int(np.sum(2 * np.asarray(ao_l) + 1))
    opt = N.Options(float(schwarz_thresh), 0, 0)
    Cin = arr(C, np.float64) if C is not None else None
    Din = arr(D, np.float64) if D is not None else None
    nocc = Cin.shape[1] if Cin is not None else 0
    J = np.zeros((nao, nao))
    K = np.zeros((nao, nao))
    E = np.zeros(2)
    nul = ctypes.POINTER(ctypes.c_double)()
    _check(N.lib().dfjk_build_host(len(xyz), xyz.ctypes.data_as(N.P_dbl), ctypes.byref(ao), ctypes.byref(aux),
                                   ctypes.byref(opt), Cin.ctypes.data_as(N.P_dbl) if Cin is not None else nul,
                                   int(nocc), Din.ctypes.data_as(N.P_dbl) if Din is not None else nul,
                                   PRECISION[precision], J.ctypes.data_as(N.P_dbl), K.ctypes.data_as(N.P_dbl),
                                   E.ctypes.data_as(N.P_dbl)))
    return J, K, E


def boys(mmax, T, stream=None):
    """F_0..F_mmax at the points T (CUDA float64 tensor) with the device routine."""
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    F = torch.empty((T.numel(), mmax + 1), dtype=torch.float64, device="cuda")
    _check(N.lib().dfjk_boys(int(mmax), T.numel(), _ptr(T), _ptr(F), _stream_handle(stream)))
    return F
