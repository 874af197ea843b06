"""Particle sets backed by torch device memory.

A ParticleSet owns one torch tensor per (property, component) -- the SoA
copy -- and one uint8 tensor of records -- the AoS copy -- and binds them to
the library with soax_bind.  Every operation runs in the library's kernels
on the current torch stream; this module only marshals arguments.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

TORCH_DTYPE = {"i8": torch.int8, "u8": torch.uint8, "i32": torch.int32, "i64": torch.int64,
               "f32": torch.float32, "f64": torch.float64}
NUMPY_DTYPE = {"i8": np.int8, "u8": np.uint8, "i32": np.int32, "i64": np.int64,
               "f32": np.float32, "f64": np.float64}


MAX_PARTICLES = 2 ** 31 - 1  # records a set can hold (the C ABI's limit)


def current_stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def params(abc=None, wrap=False):
    a = (0.0, 0.0, 0.0) if abc is None else tuple(float(v) for v in abc)
    return _lib.Params(a[0], a[1], a[2], int(bool(wrap)))


class Schema:
    """An ordered list of (name, dtype, dim[, tag]) properties."""

    def __init__(self, fields, packed=False):
        self.fields = [tuple(f) for f in fields]
        self.packed = bool(packed)
        self._c, self._keep = _lib.make_schema(self.fields, self.packed)

    @property
    def ref(self):
        return ctypes.byref(self._c)

    def layout(self):
        """(AoS field offsets, AoS record stride, SoA bytes per particle)."""
        off = (ctypes.c_int64 * len(self.fields))()
        stride, soa = ctypes.c_int64(), ctypes.c_int64()
        check(lib().soax_schema_layout(self.ref, off, ctypes.byref(stride), ctypes.byref(soa)),
              "soax_schema_layout")
        return list(off), stride.value, soa.value

    def arrays(self):
        return [(f[0], c, f[1]) for f in self.fields for c in range(int(f[2]))]

    def array_index(self, name, comp=0):
        a = 0
        for f in self.fields:
            if f[0] == name:
                return a + comp
            a += int(f[2])
        raise KeyError(name)


class ParticleSet:
    """n particles of a schema, both layouts resident on the current GPU.

    The buffers hold `capacity` >= n particles; resize and push_back grow
    them (to at least twice the capacity) through the library, which copies
    the particles into the new buffers."""

    def __init__(self, fields, n, packed=False, soa=True, aos=True, pad=64, capacity=None,
                 aosoa=False):
        if not torch.cuda.is_available():
            raise RuntimeError("ParticleSet needs a GPU")
        self.schema = Schema(fields, packed)
        self.n = int(n)
        self.pad = int(pad)
        self.offsets, self.stride, self.soa_bytes = self.schema.layout()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._has_soa, self._has_aos = bool(soa), bool(aos)
        cap = max(self.n, int(capacity or 0))
        self._alloc(cap)
        h = ctypes.c_void_p()
        check(lib().soax_bind_capacity(self.schema.ref, self.n, self.capacity, self._soa_ptrs(),
                                       self._aos_ptr(), ctypes.byref(h)), "soax_bind_capacity")
        self.handle = h
        self._aosoa_store = None
        if aosoa:
            self._bind_aosoa()
        self._views()

    # --------------------------------------------------------------- storage
    def _bind_aosoa(self):
        """Allocate and attach a tiled (AoSoA) copy sized for the capacity."""
        tile = ctypes.c_int64()
        check(lib().soax_aosoa_layout(self.schema.ref, None, ctypes.byref(tile)),
              "soax_aosoa_layout")
        nbytes = max(-(-self.capacity // 64) * tile.value, 16)
        self._aosoa_store = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
        check(lib().soax_bind_aosoa(self.handle, ctypes.c_void_p(self._aosoa_store.data_ptr()),
                                    nbytes), "soax_bind_aosoa")
        self.aosoa_tile_bytes = tile.value

    def _alloc(self, cap):
        ld = max(self.pad, -(-cap // self.pad) * self.pad)
        self.capacity = min(ld, MAX_PARTICLES)  # the buffers' whole length, up to the limit
        self._soa_store = [torch.empty(ld, dtype=TORCH_DTYPE[t], device=self.device)
                           for _, _, t in self.schema.arrays()] if self._has_soa else None
        self._aos_store = torch.zeros(max(ld * self.stride, 16), dtype=torch.uint8,
                                      device=self.device) if self._has_aos else None

    def _soa_ptrs(self):
        if not self._has_soa:
            return None
        return (ctypes.c_void_p * len(self._soa_store))(*[t.data_ptr() for t in self._soa_store])

    def _aos_ptr(self):
        return ctypes.c_void_p(self._aos_store.data_ptr()) if self._has_aos else None

    def _views(self):
        n = ctypes.c_int64()
        check(lib().soax_capacity(self.handle, ctypes.byref(n), None), "soax_capacity")
        self.n = n.value
        self.soa = [b[: self.n] for b in self._soa_store] if self._has_soa else None
        self.aos = self._aos_store if self._has_aos else None

    def _ensure(self, need):
        if need <= self.capacity:
            return
        old = (self._soa_store, self._aos_store)
        self._alloc(min(max(need, 2 * self.capacity), MAX_PARTICLES))
        check(lib().soax_rebind(self.handle, self.capacity, self._soa_ptrs(), self._aos_ptr(),
                                current_stream()), "soax_rebind")
        del old  # the library has copied the particles and synchronised
        if self._aosoa_store is not None:  # the move detached it; attach a larger one
            self._bind_aosoa()

    # -------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().soax_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ containers
    def resize(self, n):
        """New size; particles beyond the old size are zero bytes."""
        self._ensure(int(n))
        check(lib().soax_resize(self.handle, int(n), current_stream()), "soax_resize")
        self._views()

    def reserve(self, capacity):
        self._ensure(int(capacity))

    def push_back(self, records):
        """Append AoS-form records (bytes or a uint8 array of count * stride)."""
        buf = np.ascontiguousarray(np.frombuffer(bytes(records), np.uint8)
                                   if isinstance(records, (bytes, bytearray)) else records,
                                   dtype=np.uint8)
        if buf.size % self.stride:
            raise ValueError(f"{buf.size} bytes is not a whole number of {self.stride}-byte records")
        count = buf.size // self.stride
        self._ensure(self.n + count)
        check(lib().soax_push_back(self.handle, buf.ctypes.data_as(ctypes.c_void_p), count,
                                   current_stream()), "soax_push_back")
        self._views()

    def record_dtype(self):
        """numpy structured dtype of one AoS record (the schema's C layout)."""
        names, formats, offsets = [], [], []
        for (name, t, d), off in zip(self.schema.fields, self.offsets):
            names.append(name)
            formats.append((NUMPY_DTYPE[t], (int(d),)) if int(d) > 1 else NUMPY_DTYPE[t])
            offsets.append(off)
        return np.dtype({"names": names, "formats": formats, "offsets": offsets,
                         "itemsize": self.stride})

    def element(self, i, layout="soa"):
        """Particle i as a structured numpy record (a copy, like getElement)."""
        return np.frombuffer(self.get_record(layout, i), dtype=self.record_dtype())[0].copy()

    def set_element(self, i, rec=None, **fields):
        """Write particle i in every copy from a record (as returned by
        element()) and/or keyword field values, e.g. set_element(7, id=42)."""
        raw = self.get_record("soa" if self._has_soa else "aos", i) if rec is None \
            else np.asarray(rec).tobytes()
        # work on the record's own bytes so that padding keeps its value
        r = np.frombuffer(bytearray(raw), dtype=self.record_dtype())
        for name, value in fields.items():
            r[name] = value
        self.set_record(i, r.tobytes())

    def set_record(self, i, record):
        buf = np.ascontiguousarray(np.frombuffer(bytes(record), np.uint8))
        if buf.size != self.stride:
            raise ValueError(f"a record is {self.stride} bytes")
        check(lib().soax_set_record(self.handle, int(i), buf.ctypes.data_as(ctypes.c_void_p)),
              "soax_set_record")

    def remove_flagged(self, flags):
        """Remove particles whose flag (a uint8 device tensor of n) is nonzero by
        overwriting them with the last particle; returns the new size."""
        if flags.dtype not in (torch.uint8, torch.bool) or not flags.is_cuda:
            raise TypeError("flags must be a uint8 or bool device tensor")
        if flags.numel() < self.n or not flags.is_contiguous():
            raise ValueError("flags must be a contiguous tensor of n elements")
        new_n = ctypes.c_int64()
        check(lib().soax_remove_flagged(self.handle, ctypes.c_void_p(flags.data_ptr()),
                                        ctypes.byref(new_n), current_stream()),
              "soax_remove_flagged")
        self._views()
        return new_n.value

    # ----------------------------------------------------------- expressions
    def arr(self, name, comp=0):
        """Array `comp` of property `name` as an expression leaf."""
        from .expr import ARRAY, Expr
        return Expr([(ARRAY, ("soa", id(self), self.schema.array_index(name, comp)), 0.0)])

    def assign(self, dst, expr):
        """SoA array dst = (name, comp) or an array index, set to the fused
        expression over this set's arrays, for all n particles."""
        from .expr import as_expr
        expr = as_expr(expr)
        d = dst if isinstance(dst, int) else self.schema.array_index(*dst)

        def index_of(key):
            if not (isinstance(key, tuple) and key[:2] == ("soa", id(self))):
                raise ValueError("the expression reads arrays of another set")
            return key[2]

        prog = expr.program(index_of)
        check(lib().soax_eval(self.handle, d, prog, len(prog), current_stream()), "soax_eval")

    # ------------------------------------------------------------ operations
    def fill(self, seed=0, vel_mode=0, abc=None):
        p = params(abc)
        check(lib().soax_fill(self.handle, seed, vel_mode, ctypes.byref(p), current_stream()),
              "soax_fill")

    def step(self, layout, integrator, dt, nsteps, abc=None, wrap=True):
        lay = _lib.LAYOUTS[layout] if isinstance(layout, str) else layout
        integ = _lib.INTEGRATORS[integrator] if isinstance(integrator, str) else integrator
        p = params(abc, wrap)
        check(lib().soax_step(self.handle, lay, integ, float(dt), int(nsteps), ctypes.byref(p),
                              current_stream()), "soax_step")

    def step_fused(self, integrator, dt, nsteps, abc=None, wrap=True):
        """nsteps SoA steps in one launch with every particle held in registers
        in between; the same results as step("soa", ...), bit for bit."""
        integ = _lib.INTEGRATORS[integrator] if isinstance(integrator, str) else integrator
        p = params(abc, wrap)
        check(lib().soax_step_fused(self.handle, integ, float(dt), int(nsteps), ctypes.byref(p),
                                    current_stream()), "soax_step_fused")

    def step_graph(self, layout, integrator, dt, nsteps, abc=None, wrap=True):
        """The nsteps launches of step() captured once; call .launch() to replay."""
        return StepGraph(self, layout, integrator, dt, nsteps, abc, wrap)

    def step_config(self, layout, block=0, per_thread=0):
        lay = _lib.LAYOUTS[layout] if isinstance(layout, str) else layout
        check(lib().soax_step_config(self.handle, lay, block, per_thread), "soax_step_config")

    def aos_to_soa(self):
        check(lib().soax_aos_to_soa(self.handle, current_stream()), "soax_aos_to_soa")

    def soa_to_aos(self):
        check(lib().soax_soa_to_aos(self.handle, current_stream()), "soax_soa_to_aos")

    def soa_to_aosoa(self):
        check(lib().soax_soa_to_aosoa(self.handle, current_stream()), "soax_soa_to_aosoa")

    def aosoa_to_soa(self):
        check(lib().soax_aosoa_to_soa(self.handle, current_stream()), "soax_aosoa_to_soa")

    def download_aosoa(self):
        """The tiled copy's bytes for the first ceil(n / 64) tiles."""
        nt = -(-self.n // 64)
        return self._aosoa_store[: nt * self.aosoa_tile_bytes].cpu().numpy()

    def get_record(self, layout, i):
        buf = (ctypes.c_uint8 * self.stride)()
        lay = _lib.LAYOUTS[layout] if isinstance(layout, str) else layout
        check(lib().soax_get_record(self.handle, lay, int(i), buf), "soax_get_record")
        return bytes(buf)

    # --------------------------------------------------------- host transfer
    def array(self, name, comp=0):
        return self.soa[self.schema.array_index(name, comp)]

    def upload_soa(self, arrays):
        for dst, src in zip(self.soa, arrays):
            dst.copy_(torch.from_numpy(np.ascontiguousarray(src)))

    def download_soa(self):
        return [t.cpu().numpy() for t in self.soa]

    def upload_aos(self, buf):
        assert self.aos is not None
        self.aos[: self.n * self.stride].copy_(torch.from_numpy(np.ascontiguousarray(buf)))

    def download_aos(self):
        return self.aos[: self.n * self.stride].cpu().numpy()


class StepGraph:
    """A captured sequence of steps of one set (soax_step_graph_*)."""

    def __init__(self, ps, layout, integrator, dt, nsteps, abc=None, wrap=True):
        lay = _lib.LAYOUTS[layout] if isinstance(layout, str) else layout
        integ = _lib.INTEGRATORS[integrator] if isinstance(integrator, str) else integrator
        p = params(abc, wrap)
        h = ctypes.c_void_p()
        check(lib().soax_step_graph_create(ps.handle, lay, integ, float(dt), int(nsteps),
                                           ctypes.byref(p), ctypes.byref(h)),
              "soax_step_graph_create")
        self.set = ps  # keeps the set alive while the graph exists
        self.handle = h

    def launch(self):
        check(lib().soax_step_graph_launch(self.handle, current_stream()), "soax_step_graph_launch")

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().soax_step_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy(dst, src):
    """dst <- src (16-byte aligned tensors of equal byte size) with the copy kernel."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    check(lib().soax_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                          nbytes, current_stream()), "soax_copy")


PROBES = {"rk2": 0, "euler": 1, "read": 2, "write": 3}


def probe(pattern, pos, vel=None):
    """One launch of a bandwidth probe (soax_probe) on three float64 position
    tensors and three float32 velocity tensors of n elements each: "rk2",
    "euler", "read" or "write"."""
    n = pos[0].numel()
    for t in pos:
        assert t.dtype == torch.float64 and t.numel() == n
    pp = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in pos])
    vp = None
    if vel is not None:
        for t in vel:
            assert t.dtype == torch.float32 and t.numel() == n
        vp = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in vel])
    check(lib().soax_probe(PROBES[pattern], pp, vp, n, current_stream()), "soax_probe")
