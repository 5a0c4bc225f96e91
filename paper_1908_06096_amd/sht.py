"""Python binding of the C-ABI library ``libshtmi.so`` (include/sht.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
The library must have been built (``python -m paper_1908_06096_amd.build``);
loading raises if it is missing -- there is no fallback path.
"""

import ctypes
import os

import numpy as np

__all__ = ["Plan", "Batch", "Stepper", "SHTError", "library", "LIB_PATH", "GRIDS", "PRECISIONS", "TILES", "exported_symbols"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libshtmi.so")
GRIDS = {"full": 0, "octahedral": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
TILES = {"c128": 0, "c64": 1, "c32": 2}
DIRECTIONS = {"inverse": 0, "direct": 1}
OPS = {"dlambda": 0, "laplacian": 1, "inv_laplacian": 2}
STATIC_SCRATCH_BYTES = 64 << 20
BATCH_PERSISTENT = 1
BATCH_GRAPH = 2

_c_int_p = ctypes.POINTER(ctypes.c_int32)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)


class SHTInfo(ctypes.Structure):
    _fields_ = [
        ("truncation", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("nfields", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("nlat", ctypes.c_int32),
        ("fpad", ctypes.c_int32),
        ("npts", ctypes.c_int64),
        ("nspec", ctypes.c_int64),
        ("nfour", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("table_bytes", ctypes.c_int64),
        ("plan_bytes", ctypes.c_int64),
        ("elem_bytes", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("own_bytes", ctypes.c_int64),
        ("vector", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("table_free", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("chunk_table_bytes", ctypes.c_int64),
    ]


_SIGNATURES = {
    "sht_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p]),
    "sht_plan_create_like": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p]),
    "sht_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sht_plan_destroy_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sht_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SHTInfo)]),
    "sht_plan_geometry": (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_int_p, _c_int_p, _c_i64_p,
                                         _c_i64_p]),
    "sht_plan_legendre_table": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_dbl_p, _c_int_p]),
    "sht_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p]),
    "sht_inverse": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "sht_direct": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "sht_legendre_inverse": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    "sht_fourier_synthesis": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    "sht_fourier_analysis": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    "sht_legendre_direct": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    "sht_plan_set_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "sht_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p]),
    "sht_batch_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p]),
    "sht_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "sht_batch_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sht_batch_direct": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sht_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sht_batch_tiles": (ctypes.c_int, [ctypes.c_void_p, _c_int_p]),
    "sht_batch_set_tiles": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, ctypes.c_void_p]),
    "sht_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sht_plan_create_vector": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "sht_plan_create_table_free": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]),
    "sht_vector_inverse": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "sht_vector_direct": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "sht_gradient": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "sht_spectral_op": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "sht_stepper_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "sht_stepper_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "sht_stepper_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sht_transform_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "sht_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sht_last_hip_error": (ctypes.c_int, []),
}

_LIB = None


def library():
    """Load libshtmi.so (once) and declare its signatures."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1908_06096_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def exported_symbols():
    """Names the binding declares (all of them are in include/sht.h)."""
    return sorted(_SIGNATURES)


class SHTError(RuntimeError):
    def __init__(self, status, call):
        lib = library()
        msg = lib.sht_strerror(status).decode()
        hip = lib.sht_last_hip_error() if status == -4 else 0
        super().__init__(f"{call}: {msg} (status {status}{', hip error %d' % hip if hip else ''})")
        self.status = status


def _check(status, call):
    if status != 0:
        raise SHTError(status, call)


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A transform plan: truncation N, grid ('full' | 'octahedral'), F fields,
    precision ('fp64' | 'fp32' | 'bf16x3').  Tables are computed on the GPU at
    creation and stay resident until ``close()``.  With ``vector=True`` the
    plan serves F vector fields (vorticity / divergence <-> winds, gradients)
    instead of scalar transforms."""

    def __init__(self, truncation, grid="full", nfields=1, precision="fp64", stream=None, like=None, vector=False,
                 table_free=False, chunk_bytes=0):
        lib = library()
        self._lib = lib
        self._h = ctypes.c_void_p()
        if like is not None:
            # same tables as `like`, another field count
            truncation, grid, precision, vector = like.truncation, like.grid, like.precision, like.vector
            _check(lib.sht_plan_create_like(ctypes.byref(self._h), like._h, int(nfields), _stream_handle(stream)),
                   "sht_plan_create_like")
        else:
            args = [ctypes.byref(self._h), int(truncation), GRIDS[grid], int(nfields), PRECISIONS[precision]]
            if table_free:
                name = "sht_plan_create_table_free"
                args.append(ctypes.c_size_t(int(chunk_bytes)))
            else:
                name = "sht_plan_create_vector" if vector else "sht_plan_create"
            _check(getattr(lib, name)(*args, _stream_handle(stream)), name)
        self.vector = bool(vector)
        self.table_free = bool(table_free) if like is None else like.table_free
        info = SHTInfo()
        _check(lib.sht_plan_info(self._h, ctypes.byref(info)), "sht_plan_info")
        self.info = info
        self.truncation = int(truncation)
        self.grid = grid
        self.nfields = int(nfields)
        self.precision = precision
        self.nlat = info.nlat
        self.npts = info.npts
        self.nspec = info.nspec
        self.nfour = info.nfour
        self.fpad = info.fpad

    # ---- lifetime ----
    def close(self):
        if self._h:
            _check(self._lib.sht_plan_destroy(self._h), "sht_plan_destroy")
            self._h = ctypes.c_void_p()

    def close_async(self, stream):
        """Release in stream order on ``stream`` without synchronising the
        device; no work on other streams may still use the plan."""
        if self._h:
            _check(self._lib.sht_plan_destroy_async(self._h, _stream_handle(stream)), "sht_plan_destroy_async")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- metadata ----
    @property
    def dtype(self):
        import torch

        return torch.float64 if self.precision == "fp64" else torch.float32

    @property
    def workspace_bytes(self):
        return int(self._lib.sht_workspace_size(self._h))

    def geometry(self):
        n = self.nlat
        mu = np.zeros(n)
        w = np.zeros(n)
        nlon = np.zeros(n, dtype=np.int32)
        mmax = np.zeros(n, dtype=np.int32)
        off = np.zeros(n + 1, dtype=np.int64)
        frow = np.zeros(n + 1, dtype=np.int64)
        _check(self._lib.sht_plan_geometry(self._h, mu.ctypes.data_as(_c_dbl_p), w.ctypes.data_as(_c_dbl_p),
                                           nlon.ctypes.data_as(_c_int_p), mmax.ctypes.data_as(_c_int_p),
                                           off.ctypes.data_as(_c_i64_p), frow.ctypes.data_as(_c_i64_p)),
               "sht_plan_geometry")
        return {"mu": mu, "w": w, "nlon": nlon, "mmax": mmax, "ring_offset": off, "four_row": frow}

    @property
    def tile(self):
        info = SHTInfo()
        _check(self._lib.sht_plan_info(self._h, ctypes.byref(info)), "sht_plan_info")
        return {v: k for k, v in TILES.items()}[info.tile]

    def set_tile(self, tile, stream=None):
        _check(self._lib.sht_plan_set_tile(self._h, TILES[tile], _stream_handle(stream)), "sht_plan_set_tile")

    def legendre_table(self, m):
        first = ctypes.c_int32()
        _check(self._lib.sht_plan_legendre_table(self._h, int(m), None, ctypes.byref(first)),
               "sht_plan_legendre_table")
        rows = self.nlat // 2 - first.value
        out = np.zeros((rows, self.truncation - m + 1))
        if out.size:
            _check(self._lib.sht_plan_legendre_table(self._h, int(m), out.ctypes.data_as(_c_dbl_p),
                                                     ctypes.byref(first)), "sht_plan_legendre_table")
        return first.value, out

    # ---- buffers ----
    def empty_spec(self, device="cuda"):
        import torch

        return torch.empty((self.nfields, self.nspec, 2), dtype=self.dtype, device=device)

    def empty_grid(self, device="cuda"):
        import torch

        return torch.empty((self.nfields, self.npts), dtype=self.dtype, device=device)

    def empty_workspace(self, device="cuda"):
        import torch

        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def _ptr(self, t, numel, name, dtype=None):
        import torch

        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        want = self.dtype if dtype is None else dtype
        if t.dtype != want:
            raise TypeError(f"{name} must be {want}, got {t.dtype}")
        if t.numel() < numel:
            raise ValueError(f"{name} too small: {t.numel()} < {numel}")
        if t.data_ptr() % 16:
            raise ValueError(f"{name} must be 16-byte aligned")
        return ctypes.c_void_p(t.data_ptr())

    def _spec(self, t):
        return self._ptr(t, self.nfields * self.nspec * 2, "spec")

    def _grid(self, t):
        return self._ptr(t, self.nfields * self.npts, "grid")

    def empty_vortdiv(self, device="cuda"):
        """[2, F, nspec, 2]: vorticity fields, then divergence fields."""
        import torch

        return torch.empty((2, self.nfields, self.nspec, 2), dtype=self.dtype, device=device)

    def empty_uv(self, device="cuda"):
        """[2, F, npts]: U = u cos(lat) fields, then V = v cos(lat) fields."""
        import torch

        return torch.empty((2, self.nfields, self.npts), dtype=self.dtype, device=device)

    def _vortdiv(self, t):
        return self._ptr(t, 2 * self.nfields * self.nspec * 2, "vortdiv")

    def _uv(self, t):
        return self._ptr(t, 2 * self.nfields * self.npts, "uv")

    def _ws(self, t):
        import torch

        return self._ptr(t, self.workspace_bytes, "workspace", dtype=torch.uint8)

    # ---- transforms ----
    def _temporaries(self, stream, device, **make):
        """Buffers the caller did not pass, allocated on the stream the
        library will use (so the caching allocator does not hand them to
        other streams' work while the kernels still run)."""
        import torch

        st = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            return {k: f(device) for k, f in make.items()}

    def inverse(self, spec, grid=None, workspace=None, stream=None):
        """Synthesis spectral -> grid, enqueued on ``stream`` (default: the
        current stream)."""
        tmp = {}
        if grid is None:
            tmp["grid"] = self.empty_grid
        if workspace is None:
            tmp["ws"] = self.empty_workspace
        t = self._temporaries(stream, spec.device, **tmp) if tmp else {}
        grid = t.get("grid", grid)
        workspace = t.get("ws", workspace)
        _check(self._lib.sht_inverse(self._h, self._spec(spec), self._grid(grid), self._ws(workspace),
                                     _stream_handle(stream)), "sht_inverse")
        return grid

    def direct(self, grid, spec=None, workspace=None, stream=None):
        """Analysis grid -> spectral, enqueued on ``stream`` (default: the
        current stream)."""
        tmp = {}
        if spec is None:
            tmp["spec"] = self.empty_spec
        if workspace is None:
            tmp["ws"] = self.empty_workspace
        t = self._temporaries(stream, grid.device, **tmp) if tmp else {}
        spec = t.get("spec", spec)
        workspace = t.get("ws", workspace)
        _check(self._lib.sht_direct(self._h, self._grid(grid), self._spec(spec), self._ws(workspace),
                                    _stream_handle(stream)), "sht_direct")
        return spec

    def transform_static(self, direction, x, out, stream=None):
        """``inverse`` (x = spec, out = grid) or ``direct`` (x = grid, out =
        spec) with the library's per-device static scratch as the workspace:
        allocates nothing.  Calls that overlap on one GPU race."""
        if direction == "inverse":
            a, b = self._spec(x), self._grid(out)
        else:
            a, b = self._grid(x), self._spec(out)
        _check(self._lib.sht_transform_static(self._h, DIRECTIONS[direction], a, b, _stream_handle(stream)),
               "sht_transform_static")
        return out

    # ---- derivatives and vector transforms (vector plans) ----
    def _run(self, fn, name, x, out, make_out, workspace, stream):
        tmp = {}
        if out is None:
            tmp["out"] = make_out
        if workspace is None:
            tmp["ws"] = self.empty_workspace
        t = self._temporaries(stream, x.device, **tmp) if tmp else {}
        out = t.get("out", out)
        workspace = t.get("ws", workspace)
        a, b = fn(x, out)
        _check(getattr(self._lib, name)(self._h, a, b, self._ws(workspace), _stream_handle(stream)), name)
        return out

    def vector_inverse(self, vortdiv, uv=None, workspace=None, stream=None):
        """Winds [2, F, npts] (U, V) from vorticity and divergence [2, F, nspec, 2]."""
        return self._run(lambda x, o: (self._vortdiv(x), self._uv(o)), "sht_vector_inverse", vortdiv, uv,
                         self.empty_uv, workspace, stream)

    def vector_direct(self, uv, vortdiv=None, workspace=None, stream=None):
        """Vorticity and divergence [2, F, nspec, 2] from winds [2, F, npts]."""
        return self._run(lambda x, o: (self._uv(x), self._vortdiv(o)), "sht_vector_direct", uv, vortdiv,
                         self.empty_vortdiv, workspace, stream)

    def gradient(self, spec, uv=None, workspace=None, stream=None):
        """(df/dlambda, (1 - mu^2) df/dmu) [2, F, npts] of scalar fields [F, nspec, 2]."""
        return self._run(lambda x, o: (self._spec(x), self._uv(o)), "sht_gradient", spec, uv, self.empty_uv,
                         workspace, stream)

    def spectral_op(self, op, x, out=None, stream=None):
        """``dlambda`` | ``laplacian`` | ``inv_laplacian`` on spectral fields
        [..., nspec, 2] of the plan's truncation (out may be x)."""
        import torch

        count = x.numel() // (self.nspec * 2)
        if count * self.nspec * 2 != x.numel():
            raise ValueError("x must hold whole spectral fields")
        if out is None:
            with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
                out = torch.empty_like(x)
        a = self._ptr(x, count * self.nspec * 2, "x")
        b = self._ptr(out, count * self.nspec * 2, "out")
        _check(self._lib.sht_spectral_op(self._h, OPS[op], count, a, b, _stream_handle(stream)), "sht_spectral_op")
        return out

    def legendre_inverse(self, spec, workspace, stream=None):
        _check(self._lib.sht_legendre_inverse(self._h, self._spec(spec), self._ws(workspace),
                                              _stream_handle(stream)), "sht_legendre_inverse")
        return workspace

    def fourier_synthesis(self, workspace, grid, stream=None):
        _check(self._lib.sht_fourier_synthesis(self._h, self._ws(workspace), self._grid(grid),
                                               _stream_handle(stream)), "sht_fourier_synthesis")
        return grid

    def fourier_analysis(self, grid, workspace, stream=None):
        _check(self._lib.sht_fourier_analysis(self._h, self._grid(grid), self._ws(workspace),
                                              _stream_handle(stream)), "sht_fourier_analysis")
        return workspace

    def legendre_direct(self, workspace, spec, stream=None):
        _check(self._lib.sht_legendre_direct(self._h, self._ws(workspace), self._spec(spec),
                                             _stream_handle(stream)), "sht_legendre_direct")
        return spec

    # ---- workspace views (documented layouts of include/sht.h) ----
    def synthesis_fourier_view(self, workspace):
        """Complex view [nfour, fpad] of the synthesis-form workspace."""
        import torch

        t = workspace[: self.nfour * self.fpad * 2 * self.info.elem_bytes].view(self.dtype)
        return torch.view_as_complex(t.view(self.nfour, self.fpad, 2))

    def analysis_fourier_view(self, workspace):
        """Complex view [nfour/2, 2, fpad] of the analysis-form workspace (row
        index four_row[j] + m for north ring j; slot 0 the scaled
        coefficients of ring j, slot 1 those of its mirror ring)."""
        import torch

        t = workspace[: self.nfour * self.fpad * 2 * self.info.elem_bytes].view(self.dtype)
        return torch.view_as_complex(t.view(self.nfour // 2, 2, self.fpad, 2))


class Batch:
    """Several plans of one precision run in shared launches.  ``bind`` the
    device buffers of every transform, then ``inverse`` / ``direct`` enqueue
    all of them on the stream; ``tune`` picks each plan's tile variant by
    timing."""

    def __init__(self, plans, persistent=True, graph=False, stream=None):
        lib = library()
        self._lib = lib
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        self._h = ctypes.c_void_p()
        flags = (BATCH_PERSISTENT if persistent else 0) | (BATCH_GRAPH if graph else 0)
        _check(lib.sht_batch_create(ctypes.byref(self._h), arr, len(self.plans), flags, _stream_handle(stream)),
               "sht_batch_create")
        self._bound = None

    @property
    def workspace_bytes(self):
        return int(self._lib.sht_batch_workspace_size(self._h))

    def bind(self, specs, grids, workspace=None, stream=None):
        """Bind every transform's buffers, in stream order on ``stream``
        (default: the current stream)."""
        import torch

        if workspace is None:
            with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
                workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")
        n = len(self.plans)
        sp = (ctypes.c_void_p * n)(*[p._spec(s).value for p, s in zip(self.plans, specs)])
        gp = (ctypes.c_void_p * n)(*[p._grid(g).value for p, g in zip(self.plans, grids)])
        if workspace.numel() < self.workspace_bytes or workspace.dtype != torch.uint8:
            raise ValueError("workspace too small")
        _check(self._lib.sht_batch_bind(self._h, sp, gp, ctypes.c_void_p(workspace.data_ptr()),
                                        _stream_handle(stream)), "sht_batch_bind")
        self._bound = (list(specs), list(grids), workspace)
        return workspace

    def inverse(self, stream=None):
        _check(self._lib.sht_batch_inverse(self._h, _stream_handle(stream)), "sht_batch_inverse")

    def direct(self, stream=None):
        _check(self._lib.sht_batch_direct(self._h, _stream_handle(stream)), "sht_batch_direct")

    def tune(self, stream=None, cache=None):
        """Pick each plan's tile variant by timing (sht_batch_tune).  With
        ``cache`` (a JSON file path), choices made before on this device for
        the same (truncation, grid, fields, precision) are applied without
        timing, and new ones are added to the file."""
        import json

        if cache is None:
            _check(self._lib.sht_batch_tune(self._h, _stream_handle(stream)), "sht_batch_tune")
            return self.tiles()
        import torch

        dev = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = getattr(dev, "gcnArchName", dev.name)
        keys = [f"{arch}|T{p.truncation}|{p.grid}|F{p.nfields}|{p.precision}" for p in self.plans]
        try:
            with open(cache) as fh:
                known = json.load(fh)
        except (OSError, ValueError):
            known = {}
        if all(k in known for k in keys):
            tiles = (ctypes.c_int32 * len(self.plans))(*[TILES[known[k]] for k in keys])
            _check(self._lib.sht_batch_set_tiles(self._h, tiles, _stream_handle(stream)), "sht_batch_set_tiles")
            return self.tiles()
        _check(self._lib.sht_batch_tune(self._h, _stream_handle(stream)), "sht_batch_tune")
        chosen = self.tiles()
        known.update(dict(zip(keys, chosen)))
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(known, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
        return chosen

    def set_tiles(self, tiles, stream=None):
        arr = (ctypes.c_int32 * len(self.plans))(*[TILES[t] for t in tiles])
        _check(self._lib.sht_batch_set_tiles(self._h, arr, _stream_handle(stream)), "sht_batch_set_tiles")

    def tiles(self):
        out = (ctypes.c_int32 * len(self.plans))()
        _check(self._lib.sht_batch_tiles(self._h, out), "sht_batch_tiles")
        inv = {v: k for k, v in TILES.items()}
        return [inv[x] for x in out]

    def close(self):
        if self._h:
            _check(self._lib.sht_batch_destroy(self._h), "sht_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Stepper:
    """Time steps of du/dt = nu Lap u + r u (1 - u) on the unit sphere
    (semi-implicit Euler: logistic term on the grid, implicit diffusion in
    spectral space) on a scalar plan.  ``spec`` [F, nspec, 2] is the state,
    updated in place by ``run``; ``graph=True`` captures ``graph_steps``
    steps into a HIP graph (on ``stream``, which must not be the null
    stream) and replays it."""

    def __init__(self, plan, spec, dt, rate, nu, graph=False, graph_steps=1, grid=None, workspace=None,
                 stream=None):
        import torch

        self._lib = plan._lib
        self.plan = plan
        st = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            self.grid = plan.empty_grid() if grid is None else grid
            self.workspace = plan.empty_workspace() if workspace is None else workspace
        self.spec = spec
        self._h = ctypes.c_void_p()
        _check(self._lib.sht_stepper_create(ctypes.byref(self._h), plan._h, float(dt), float(rate), float(nu),
                                            plan._spec(spec), plan._grid(self.grid), plan._ws(self.workspace),
                                            1 if graph else 0, int(graph_steps), _stream_handle(st)),
               "sht_stepper_create")

    def run(self, nsteps, stream=None):
        _check(self._lib.sht_stepper_run(self._h, int(nsteps), _stream_handle(stream)), "sht_stepper_run")

    def close(self):
        if self._h:
            _check(self._lib.sht_stepper_destroy(self._h), "sht_stepper_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
