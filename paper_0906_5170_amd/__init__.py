"""Python binding of the MI355X Casimir-force FDTD library (libcasimir_fdtd.so).

Argument marshalling only: every step of the force solve runs in the HIP
library behind the C ABI of include/casimir_fdtd.h.  PyTorch provides the
device workspace (a uint8 tensor) and the stream.  Loading fails loudly when
the built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcasimir_fdtd.so")

COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
BC = {"pec": 0, "periodic": 1, "pml": 2}
POL = {"TM": 1, "TE": 2, "TM+TE": 3, "3D": 4}
KERNEL = {"general": 0, "zinv2d": 1}
PRECISION = {"fp64": 0, "fp32": 1}
PATH = {"batched": 0, "plain": 1}
COORD = {"cartesian": 0, "cylindrical": 1, "kz": 2}
FLAG_KEEP_GAMMA = 1
FLAG_TIME_STENCIL = 2
FLAG_SPLIT = 4
FLAG_INJECT_NAN = 8
FLAG_GRAPH = 16
STATUS = {0: "CF_OK", 1: "CF_E_ARG", 2: "CF_E_CFL", 3: "CF_E_SURFACE", 4: "CF_E_BUDGET",
          5: "CF_E_NONFINITE", 6: "CF_E_DEVICE", 7: "CF_E_CANCELLED", 8: "CF_E_UNSUPPORTED"}


class CfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("res", C.c_double), ("bc", C.c_int * 3),
                ("pml_cells", C.c_int * 3), ("coord", C.c_int)]


class _Materials(C.Structure):
    _fields_ = [("n_materials", C.c_int), ("eps", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("comp_id", C.c_void_p * 6),
                ("n_lorentz", C.c_int), ("lorentz_deps", C.POINTER(C.c_double)),
                ("lorentz_w0", C.POINTER(C.c_double))]


class _Surface(C.Structure):
    _fields_ = [("lo", C.c_int * 3), ("hi", C.c_int * 3), ("n_harm", C.c_int),
                ("force_axis", C.c_int), ("m_max", C.c_int), ("kz", C.POINTER(C.c_double)),
                ("kz_weight", C.POINTER(C.c_double)), ("n_kz", C.c_int), ("kx", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("sigma", C.c_double), ("courant", C.c_double), ("n_steps", C.c_int),
                ("pol", C.c_int), ("kernel", C.c_int), ("precision", C.c_int), ("path", C.c_int),
                ("flags", C.c_int), ("channel_subset", C.POINTER(C.c_int)), ("n_subset", C.c_int),
                ("stream", C.c_void_p), ("max_resident", C.c_int), ("tile_variant", C.c_int),
                ("stop_tol", C.c_double), ("stop_every", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("n_channels", C.c_int), ("n_faces", C.c_int), ("per_harmonic_len", C.c_int),
                ("n_comp", C.c_int), ("workspace_bytes", C.c_size_t), ("eps_s", C.c_double),
                ("mu_s", C.c_double), ("n_steps_max", C.c_int)]


class _Result(C.Structure):
    _fields_ = [("force", C.c_double),
                ("per_harmonic", C.POINTER(C.c_double)), ("per_harmonic_len", C.c_int),
                ("per_face", C.POINTER(C.c_double)), ("per_face_len", C.c_int),
                ("per_channel", C.POINTER(C.c_double)), ("per_channel_len", C.c_int),
                ("gamma", C.POINTER(C.c_double)), ("gamma_len", C.c_longlong),
                ("trace", C.POINTER(C.c_double)), ("trace_len", C.c_int),
                ("n_channels_run", C.c_int), ("cell_updates", C.c_double),
                ("device_ms", C.c_double), ("stencil_ms_avg", C.c_double),
                ("stencil_samples", C.c_int), ("stencil_launches", C.c_int),
                ("stencil_alg_bytes", C.c_double), ("stencil_cell_updates", C.c_double),
                ("fused", C.c_int), ("tile_variant", C.c_int), ("tile_halo", C.c_int),
                ("n_steps_run", C.c_int), ("advanced_cell_updates", C.c_double)]


_lib = None

EXPORTS = ("cf_problem_create", "cf_problem_destroy", "cf_problem_info", "cf_channel_table",
           "cf_validate", "cf_workspace_size", "cf_solve", "cf_kernel_table", "cf_last_error",
           "cf_batch_workspace_size", "cf_batch_solve", "cf_server_create", "cf_server_submit",
           "cf_server_poll", "cf_server_wait", "cf_server_cancel", "cf_server_times", "cf_server_stats",
           "cf_server_destroy", "cf_solve_static")

# bytes of the device array cf_solve_static takes its workspace from
STATIC_WORKSPACE_BYTES = 64 << 20


def load():
    """Load the built HIP library (raises if it has not been built).

    PyTorch is imported first: its HIP runtime has the same soname
    (libamdhip64.so.7) as the one the library links, so the dynamic linker
    binds the library to PyTorch's already loaded runtime and the process
    holds a single HIP runtime (device memory and streams from PyTorch are
    then valid inside the library)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    import torch  # noqa: F401  (see docstring)
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.cf_last_error.restype = C.c_char_p
    lib.cf_problem_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Materials), C.POINTER(_Surface),
                                      C.POINTER(P)]
    lib.cf_problem_destroy.argtypes = [P]
    lib.cf_problem_info.argtypes = [P, C.POINTER(_Opts), C.POINTER(_Info)]
    lib.cf_channel_table.argtypes = [P, C.POINTER(_Opts), C.c_int] + [C.c_void_p] * 6
    lib.cf_validate.argtypes = [P, C.POINTER(_Opts)]
    lib.cf_workspace_size.argtypes = [P, C.POINTER(_Opts), C.POINTER(C.c_size_t)]
    lib.cf_solve.argtypes = [P, C.POINTER(_Opts), C.c_void_p, C.c_size_t, C.POINTER(_Result)]
    lib.cf_solve_static.argtypes = [P, C.POINTER(_Opts), C.POINTER(_Result)]
    lib.cf_kernel_table.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_double)]
    lib.cf_batch_workspace_size.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(_Opts),
                                            C.POINTER(C.c_size_t)]
    lib.cf_batch_solve.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(_Opts), C.c_void_p, C.c_size_t,
                                   C.POINTER(_Result)]
    lib.cf_server_create.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.POINTER(P)]
    lib.cf_server_submit.argtypes = [P, P, C.POINTER(_Opts), C.POINTER(C.c_uint64)]
    lib.cf_server_poll.argtypes = [P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(_Result)]
    lib.cf_server_wait.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(C.c_int), C.POINTER(_Result)]
    lib.cf_server_cancel.argtypes = [P, C.c_uint64]
    lib.cf_server_times.argtypes = [P, C.c_uint64] + [C.POINTER(C.c_double)] * 3
    lib.cf_server_stats.argtypes = [P, C.POINTER(_ServerInfo)]
    lib.cf_server_destroy.argtypes = [P]
    for name in EXPORTS:
        getattr(lib, name).restype = C.c_int if name != "cf_last_error" else C.c_char_p
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        raise CfError(code, load().cf_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _result_buffers(n_harm: int, n_chan: int, n_steps_gamma: int = 0):
    """A cf_result whose output arrays point at fresh NumPy buffers."""
    ph = np.zeros(max(1, n_harm))
    pf = np.zeros(6)
    pc = np.zeros(n_chan)
    r = _Result()
    r.per_harmonic, r.per_harmonic_len = _dptr(ph), len(ph)
    r.per_face, r.per_face_len = _dptr(pf), 6
    r.per_channel, r.per_channel_len = _dptr(pc), n_chan
    bufs = dict(ph=ph, n_harm=n_harm, pf=pf, pc=pc, gam=None, tr=None)
    if n_steps_gamma:
        bufs["gam"] = np.zeros(n_steps_gamma * n_chan)
        bufs["tr"] = np.zeros(n_steps_gamma)
        r.gamma, r.gamma_len = _dptr(bufs["gam"]), bufs["gam"].size
        r.trace, r.trace_len = _dptr(bufs["tr"]), n_steps_gamma
        bufs["T"] = n_steps_gamma
    return r, bufs


def _result_dict(r, bufs) -> dict:
    out = dict(force=r.force, per_harmonic=bufs["ph"][:bufs["n_harm"]], per_face=bufs["pf"],
               per_channel=bufs["pc"], n_channels=r.n_channels_run, cell_updates=r.cell_updates,
               device_ms=r.device_ms, stencil_ms_avg=r.stencil_ms_avg,
               stencil_samples=r.stencil_samples, stencil_launches=r.stencil_launches,
               stencil_alg_bytes=r.stencil_alg_bytes,
               stencil_cell_updates=r.stencil_cell_updates, fused=bool(r.fused),
               tile_variant=r.tile_variant, tile_halo=r.tile_halo, n_steps_run=r.n_steps_run,
               advanced_cell_updates=r.advanced_cell_updates)
    if bufs["gam"] is not None:
        out["gamma"] = bufs["gam"].reshape(bufs["T"], len(bufs["pc"]))
        out["trace"] = bufs["tr"]
    return out


def kernel_table(kernel: str, sigma: float, dt: float, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(load().cf_kernel_table(KERNEL[kernel], float(sigma), float(dt), int(n), _dptr(out)))
    return out


class Problem:
    """A force-solve problem: grid, per-component materials and the stress
    surface.  Inputs are copied by the library at construction."""

    def __init__(self, ndim: int, shape: Sequence[int], res: float, bc: Sequence[str],
                 eps: Sequence[float], mu: Sequence[float], comp_ids: Dict[str, np.ndarray],
                 s_lo: Sequence[int], s_hi: Sequence[int], n_harm: int, force_axis: int,
                 pml_cells: Sequence[int] = (0, 0, 0), coord: str = "cartesian", m_max: int = 0,
                 kz: Sequence[float] = (), kz_weight: Sequence[float] = (), kx: Sequence[float] = (),
                 lorentz: Optional[Dict[int, Sequence[Sequence[float]]]] = None):
        lib = load()
        g = _Grid()
        g.ndim = int(ndim)
        g.coord = COORD[coord]
        for a in range(3):
            g.n[a] = int(shape[a])
            g.bc[a] = BC[bc[a]]
            g.pml_cells[a] = int(pml_cells[a])
        g.res = float(res)
        self._eps = np.ascontiguousarray(eps, dtype=np.float64)
        self._mu = np.ascontiguousarray(mu, dtype=np.float64)
        m = _Materials()
        m.n_materials = len(self._eps)
        m.eps = _dptr(self._eps)
        m.mu = _dptr(self._mu)
        # Lorentz terms {id: ((d_eps, w0), ...)} as n_materials x n_terms arrays
        terms = {int(k): list(v) for k, v in (lorentz or {}).items() if v}
        n_lor = max((len(v) for v in terms.values()), default=0)
        if n_lor:
            self._lde = np.zeros((len(self._eps), n_lor))
            self._lw0 = np.zeros((len(self._eps), n_lor))
            for k, v in terms.items():
                for j, (de, w0) in enumerate(v):
                    self._lde[k, j], self._lw0[k, j] = float(de), float(w0)
            m.n_lorentz = n_lor
            m.lorentz_deps = _dptr(self._lde)
            m.lorentz_w0 = _dptr(self._lw0)
        self._ids = []
        for k, name in enumerate(COMPONENTS):
            arr = comp_ids.get(name)
            if arr is None:
                m.comp_id[k] = None
                continue
            arr = np.ascontiguousarray(arr, dtype=np.uint8)
            if arr.size != int(shape[0]) * int(shape[1]) * int(shape[2]):
                raise ValueError(f"{name} id grid has {arr.size} cells")
            self._ids.append(arr)
            m.comp_id[k] = arr.ctypes.data
        s = _Surface()
        for a in range(3):
            s.lo[a] = int(s_lo[a])
            s.hi[a] = int(s_hi[a])
        s.n_harm = int(n_harm)
        s.force_axis = int(force_axis)
        s.m_max = int(m_max)
        kz_arr = np.ascontiguousarray(kz, dtype=np.float64)
        kzw_arr = np.ascontiguousarray(kz_weight, dtype=np.float64)
        if len(kz_arr) != len(kzw_arr):
            raise ValueError("kz and kz_weight differ in length")
        if len(kz_arr):
            s.kz, s.kz_weight, s.n_kz = _dptr(kz_arr), _dptr(kzw_arr), len(kz_arr)
        kx_arr = np.ascontiguousarray(kx, dtype=np.float64)
        if len(kx_arr):
            if len(kx_arr) != len(kz_arr):
                raise ValueError("kx and kz differ in length")
            s.kx = _dptr(kx_arr)
        h = C.c_void_p()
        _check(lib.cf_problem_create(C.byref(g), C.byref(m), C.byref(s), C.byref(h)))
        self._h = h
        self.ndim = ndim
        self.coord = coord
        self.shape = tuple(int(v) for v in shape)
        self.res = float(res)
        self._ids = None

    @classmethod
    def from_workload(cls, wl) -> "Problem":
        return cls(wl.ndim, wl.shape, wl.res, wl.bc, wl.eps, wl.mu, wl.comp_ids, wl.s_lo, wl.s_hi,
                   wl.n_harm, wl.force_axis, wl.pml_cells, coord=wl.coord, m_max=wl.m_max,
                   kz=wl.kz, kz_weight=wl.kz_weight, kx=wl.kx, lorentz=getattr(wl, "lorentz", None))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value is not None and _lib is not None:
            _lib.cf_problem_destroy(h)
            self._h = None

    @property
    def n_cells(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def _opts(self, sigma=1.0, courant=0.5, n_steps=1000, pol="TM", kernel="zinv2d",
              precision="fp64", path="batched", keep_gamma=False, channel_subset=None, stream=None,
              time_stencil=False, split=False, max_resident=0, tile_variant=0, inject_nan=False,
              graph=False, stop_tol=0.0, stop_every=0):
        o = _Opts()
        o.sigma = float(sigma)
        o.courant = float(courant)
        o.n_steps = int(n_steps)
        o.pol = POL[pol]
        o.kernel = KERNEL[kernel]
        o.precision = PRECISION[precision]
        o.path = PATH[path]
        o.flags = ((FLAG_KEEP_GAMMA if keep_gamma else 0) | (FLAG_TIME_STENCIL if time_stencil else 0)
                   | (FLAG_SPLIT if split else 0) | (FLAG_INJECT_NAN if inject_nan else 0)
                   | (FLAG_GRAPH if graph else 0))
        if channel_subset is not None:
            sub = np.ascontiguousarray(channel_subset, dtype=np.int32)
            o.channel_subset = sub.ctypes.data_as(C.POINTER(C.c_int))
            o.n_subset = len(sub)
            self._subset_keep = sub
        else:
            o.channel_subset = None
            o.n_subset = 0
        o.stream = stream
        o.max_resident = int(max_resident)
        o.tile_variant = int(tile_variant)
        o.stop_tol = float(stop_tol)
        o.stop_every = int(stop_every)
        return o

    def info(self, **opts) -> dict:
        o = self._opts(**opts)
        inf = _Info()
        _check(load().cf_problem_info(self._h, C.byref(o), C.byref(inf)))
        return dict(n_channels=inf.n_channels, n_faces=inf.n_faces,
                    per_harmonic_len=inf.per_harmonic_len, n_comp=inf.n_comp,
                    workspace_bytes=int(inf.workspace_bytes), eps_s=inf.eps_s, mu_s=inf.mu_s,
                    n_steps_max=inf.n_steps_max)

    def validate(self, **opts):
        o = self._opts(**opts)
        _check(load().cf_validate(self._h, C.byref(o)))

    def channel_table(self, **opts) -> dict:
        n = self.info(**opts)["n_channels"]
        o = self._opts(**opts)
        face, label, kind, src, meas = (np.zeros(n, np.int32) for _ in range(5))
        sign = np.zeros(n)
        _check(load().cf_channel_table(self._h, C.byref(o), n, face.ctypes.data, label.ctypes.data,
                                       kind.ctypes.data, src.ctypes.data, meas.ctypes.data,
                                       sign.ctypes.data))
        return dict(face=face, label=label, kind=kind, src=src, meas=meas, sign=sign)

    def solve(self, workspace=None, **opts) -> dict:
        """Run the force solve on the GPU.  workspace: optional torch uint8
        CUDA tensor of at least info()['workspace_bytes'] bytes."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("cf solve needs a ROCm GPU")
        stream = torch.cuda.current_stream()
        opts = dict(opts)
        opts["stream"] = C.c_void_p(stream.cuda_stream)
        info = self.info(**{k: v for k, v in opts.items() if k != "stream"})
        nbytes = info["workspace_bytes"]
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        if workspace.numel() < nbytes:
            raise ValueError("workspace too small")
        o = self._opts(**opts)
        C_run = o.n_subset if o.n_subset > 0 else info["n_channels"]
        T = info["n_steps_max"]
        r, bufs = _result_buffers(info["per_harmonic_len"], C_run, T if opts.get("keep_gamma") else 0)
        _check(load().cf_solve(self._h, C.byref(o), C.c_void_p(workspace.data_ptr()), nbytes, C.byref(r)))
        out = _result_dict(r, bufs)
        return out

    def solve_static(self, **opts) -> dict:
        """Run the force solve through cf_solve_static: the library's fixed
        device array is the workspace, and nothing is allocated on the
        device (CF_E_BUDGET when the solve needs more than
        STATIC_WORKSPACE_BYTES)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("cf solve needs a ROCm GPU")
        opts = dict(opts)
        opts["stream"] = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        info = self.info(**{k: v for k, v in opts.items() if k != "stream"})
        o = self._opts(**opts)
        C_run = o.n_subset if o.n_subset > 0 else info["n_channels"]
        T = info["n_steps_max"]
        r, bufs = _result_buffers(info["per_harmonic_len"], C_run, T if opts.get("keep_gamma") else 0)
        _check(load().cf_solve_static(self._h, C.byref(o), C.byref(r)))
        return _result_dict(r, bufs)


def batch_solve(problems: Sequence["Problem"], workspace=None, **opts):
    """Solve several problems with the same options in one batched launch
    sequence (see cf_batch_solve).  Returns one result dict per problem."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("cf batch solve needs a ROCm GPU")
    lib = load()
    opts = dict(opts)
    opts.pop("keep_gamma", None)
    opts.pop("channel_subset", None)
    stream = torch.cuda.current_stream()
    o = problems[0]._opts(stream=C.c_void_p(stream.cuda_stream), **opts)
    n = len(problems)
    hs = (C.c_void_p * n)(*[p._h.value for p in problems])
    nbytes = C.c_size_t()
    _check(lib.cf_batch_workspace_size(hs, n, C.byref(o), C.byref(nbytes)))
    if workspace is None:
        workspace = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    if workspace.numel() < nbytes.value:
        raise ValueError("workspace too small")
    results = (_Result * n)()
    keep = []
    for k, p in enumerate(problems):
        inf = p.info(**opts)
        ph = np.zeros(max(1, inf["per_harmonic_len"]))
        pf = np.zeros(6)
        pc = np.zeros(inf["n_channels"])
        keep.append((ph, pf, pc, inf))
        r = results[k]
        r.per_harmonic, r.per_harmonic_len = _dptr(ph), len(ph)
        r.per_face, r.per_face_len = _dptr(pf), 6
        r.per_channel, r.per_channel_len = _dptr(pc), len(pc)
    _check(lib.cf_batch_solve(hs, n, C.byref(o), C.c_void_p(workspace.data_ptr()), nbytes.value, results))
    out = []
    for k in range(n):
        r = results[k]
        ph, pf, pc, inf = keep[k]
        out.append(dict(force=r.force, per_harmonic=ph[:inf["per_harmonic_len"]], per_face=pf,
                        per_channel=pc, n_channels=r.n_channels_run, cell_updates=r.cell_updates,
                        device_ms=r.device_ms, fused=bool(r.fused), tile_variant=r.tile_variant,
                        tile_halo=r.tile_halo, advanced_cell_updates=r.advanced_cell_updates))
    return out


REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class _ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("cancelled", C.c_uint64), ("queued", C.c_int), ("running", C.c_int),
                ("bytes_in_use", C.c_size_t), ("budget", C.c_size_t), ("clock_steps", C.c_int64),
                ("busy_s", C.c_double), ("steps_per_tick", C.c_int)]


class Server:
    """Continuous-batching force-solve server on the current GPU (see
    cf_server_create).  The device memory budget is one torch uint8 tensor
    handed to the library as its arena; the scheduler runs on a stream of
    its own.  The library copies each submitted problem into its request, so
    the Problem objects need not outlive their requests; the binding keeps
    them only to size the result buffers."""

    def __init__(self, budget_bytes: int, precision: str = "fp32", tile_variant: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("cf server needs a ROCm GPU")
        lib = load()
        self._arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        self.precision = precision
        h = C.c_void_p()
        _check(lib.cf_server_create(int(budget_bytes), PRECISION[precision], int(tile_variant),
                                    C.c_void_p(self._arena.data_ptr()), None, C.byref(h)))
        self._h = h
        self._reqs = {}

    def submit(self, problem: "Problem", **opts) -> int:
        opts = dict(opts)
        opts.setdefault("precision", self.precision)
        o = problem._opts(**opts)
        t = C.c_uint64()
        _check(load().cf_server_submit(self._h, problem._h, C.byref(o), C.byref(t)))
        info = problem.info(**opts)
        self._reqs[t.value] = (problem, info)
        return t.value

    def _take(self, fn, ticket, *extra):
        problem, info = self._reqs[ticket]
        r, bufs = _result_buffers(info["per_harmonic_len"], info["n_channels"])
        st = C.c_int()
        _check(fn(self._h, C.c_uint64(ticket), *extra, C.byref(st), C.byref(r)))
        state = REQ_STATE[st.value]
        return state, (_result_dict(r, bufs) if state == "done" else None)

    def poll(self, ticket: int):
        """(state, result or None)."""
        return self._take(load().cf_server_poll, ticket)

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        """Block until the request is done and return its result (raises
        CfError if it failed or was cancelled, TimeoutError on timeout)."""
        state, res = self._take(load().cf_server_wait, ticket, C.c_double(timeout))
        if state != "done":
            raise TimeoutError(f"request {ticket} still {state}")
        return res

    def cancel(self, ticket: int):
        _check(load().cf_server_cancel(self._h, C.c_uint64(ticket)))

    def times(self, ticket: int):
        """(submitted, admitted, done) on a monotonic clock, seconds."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(load().cf_server_times(self._h, C.c_uint64(ticket), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def stats(self) -> dict:
        i = _ServerInfo()
        _check(load().cf_server_stats(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _ServerInfo._fields_}

    def release(self, ticket: int):
        """Forget a request on the Python side (the library keeps its own
        copy of the problem, so this is safe at any time; the ticket can no
        longer be polled through this object afterwards)."""
        self._reqs.pop(ticket, None)

    def close(self):
        if self._h is not None:
            load().cf_server_destroy(self._h)
            self._h = None
            self._reqs.clear()
            self._arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_workload(wl, **over) -> dict:
    """Solve a casimir_inputs.Workload with its own run options."""
    p = Problem.from_workload(wl)
    opts = dict(sigma=wl.sigma, courant=wl.courant, n_steps=wl.n_steps, pol=wl.pol,
                kernel=wl.kernel, precision=wl.precision)
    opts.update(over)
    return p.solve(**opts)
