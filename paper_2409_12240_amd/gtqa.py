"""ctypes binding of libgtqa.so (include/gtqa.h), plus thin object wrappers.

Argument marshalling only: every step of the Trotter path runs in the HIP
library.  If the library is missing the binding raises; there is no fallback.
PyTorch, when available with a GPU, supplies the HIP stream and the device
allocator (its caching allocator).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgtqa.so")

GTQA_OK = 0
GTQA_WARN_BP_MAXITER = 1
GTQA_WARN_JACOBI_CAP = 2
GTQA_ERR_ARG = -1
GTQA_ERR_GRAPH = -2
GTQA_ERR_NOMEM = -3
GTQA_ERR_HIP = -4
GTQA_ERR_NUMERIC = -5
GTQA_ERR_STATE = -6
GTQA_BUSY = -7
GTQA_ERR_UNSUPPORTED = -8

GTQA_FP64 = 0
GTQA_MIXED = 1
REGAUGE = {"colour": 0, "step": 1, "never": 2, "adaptive": 3}
LAUNCH = {"direct": 0, "graph": 1}
BP_SCHEDULE = {"colour": 0, "flooding": 1}
GTQA_BP_WARM = 0
GTQA_BP_REGAUGE = 1
GTQA_BP_RANDOM = 2
GTQA_READ_FROM_VIDAL = 0
GTQA_READ_FROM_MESSAGES = 1

EXPORTED = [
    "gtqa_default_options", "gtqa_init_state", "gtqa_trotter_step", "gtqa_bp_converge",
    "gtqa_readout", "gtqa_free_state", "gtqa_footprint_bytes", "gtqa_strerror",
    "gtqa_colour_edges", "gtqa_version", "gtqa_pool_create", "gtqa_pool_admit",
    "gtqa_pool_step", "gtqa_pool_readout", "gtqa_pool_release", "gtqa_pool_free_bytes",
    "gtqa_pool_resident", "gtqa_pool_free", "gtqa_pool_profile", "gtqa_pool_profile_stages",
    "gtqa_pool_profile_read", "gtqa_pool_profile_sample", "gtqa_pool_bp_totals",
    "gtqa_vidal_residual", "gtqa_pool_residual", "gtqa_set_tuning", "gtqa_get_tuning",
    "gtqa_set_bipartition", "gtqa_entropy", "gtqa_spectral_bipartition", "gtqa_pool_set_bipartition",
    "gtqa_pool_entropy", "gtqa_sample", "gtqa_pool_sample", "gtqa_x_layer", "gtqa_pool_x_layer",
    "gtqa_set_network", "gtqa_get_network", "gtqa_pool_set_network", "gtqa_pool_get_network",
    "gtqa_bond_svd", "gtqa_bond_svd_noalloc", "gtqa_bond_svd_noalloc_max", "gtqa_pool_set_bp",
]

TUNE_KNOBS = {"su_edges_per_wave_chi4": 0, "xcd_contiguous": 1, "canon_lanes_chi4": 2}
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")

STAGES = ["simple_update", "bp_init", "bp_sweep", "bp_reduce", "canonicalise", "gauge_apply",
          "x_layer", "readout", "residual"]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class gtqa_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class gtqa_instance(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_edges", C.c_int32), ("edges", C.POINTER(C.c_int32)),
                ("J", C.POINTER(C.c_double)), ("h", C.POINTER(C.c_double)),
                ("colour", C.POINTER(C.c_uint8))]


class gtqa_options(C.Structure):
    _fields_ = [("chi", C.c_int32), ("precision", C.c_int32), ("bp_tol", C.c_double),
                ("bp_max_sweeps", C.c_int32), ("svd_rel_cutoff", C.c_double),
                ("eig_rel_cutoff", C.c_double), ("regauge_policy", C.c_int32),
                ("bp_schedule", C.c_int32), ("stream", C.c_void_p),
                ("allocator", C.POINTER(gtqa_allocator)), ("residual_max", C.c_double),
                ("launch_mode", C.c_int32)]


class gtqa_step_stats(C.Structure):
    _fields_ = [("n_regauges", C.c_int32), ("bp_sweeps", C.c_int32 * 8),
                ("bp_dist", C.c_double * 8), ("n_colours", C.c_int32),
                ("log_fidelity", C.c_double), ("max_trunc_error", C.c_double),
                ("log_fidelity_total", C.c_double), ("residual", C.c_double * 8),
                ("entropy", C.c_double)]


class gtqa_pool_options(C.Structure):
    _fields_ = [("base", gtqa_options), ("max_vertices", C.c_int64), ("max_edges", C.c_int64),
                ("max_slots", C.c_int32), ("budget_bytes", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgtqa.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgtqa.so not built ({path}); run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime under the same soname
    # (libamdhip64.so.7); whichever copy loads first serves the whole process.
    # Loading torch first makes the library run on torch's runtime, so that
    # torch's streams and allocations are native handles for it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.POINTER
    sigs = {
        "gtqa_default_options": (None, [P(gtqa_options)]),
        "gtqa_init_state": (C.c_int, [P(gtqa_instance), P(gtqa_options), P(C.c_void_p)]),
        "gtqa_trotter_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, P(gtqa_step_stats)]),
        "gtqa_bp_converge": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_uint32, C.c_uint64,
                                       P(C.c_int32), P(C.c_double)]),
        "gtqa_set_network": (C.c_int, [C.c_void_p, P(C.c_double), P(C.c_double)]),
        "gtqa_get_network": (C.c_int, [C.c_void_p, P(C.c_double), P(C.c_double)]),
        "gtqa_pool_set_network": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double)]),
        "gtqa_pool_get_network": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double)]),
        "gtqa_bond_svd": (C.c_int, [C.c_int32, C.c_int32, P(C.c_double), C.c_double, P(C.c_double),
                                    P(C.c_int32)]),
        "gtqa_bond_svd_noalloc": (C.c_int, [C.c_int32, C.c_int32, P(C.c_double), C.c_double, P(C.c_double),
                                            P(C.c_int32)]),
        "gtqa_bond_svd_noalloc_max": (C.c_int32, [C.c_int32]),
        "gtqa_pool_set_bp": (C.c_int, [C.c_void_p, C.c_double, C.c_int32]),
        "gtqa_readout": (C.c_int, [C.c_void_p, C.c_uint32, P(C.c_double), P(C.c_double),
                                   P(C.c_int8), P(C.c_double)]),
        "gtqa_free_state": (None, [C.c_void_p]),
        "gtqa_footprint_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "gtqa_strerror": (C.c_char_p, [C.c_int]),
        "gtqa_colour_edges": (C.c_int, [C.c_int32, C.c_int32, P(C.c_int32), P(C.c_uint8)]),
        "gtqa_version": (C.c_char_p, []),
        "gtqa_pool_create": (C.c_int, [P(gtqa_pool_options), P(C.c_void_p)]),
        "gtqa_pool_admit": (C.c_int, [C.c_void_p, P(gtqa_instance), P(C.c_int32)]),
        "gtqa_pool_step": (C.c_int, [C.c_void_p, P(C.c_int32), P(C.c_double), P(C.c_double),
                                     C.c_int32, P(gtqa_step_stats)]),
        "gtqa_pool_readout": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                                        P(C.c_int8), P(C.c_double)]),
        "gtqa_pool_release": (C.c_int, [C.c_void_p, C.c_int32]),
        "gtqa_pool_free_bytes": (C.c_int64, [C.c_void_p]),
        "gtqa_pool_resident": (C.c_int32, [C.c_void_p]),
        "gtqa_pool_free": (None, [C.c_void_p]),
        "gtqa_pool_profile": (C.c_int, [C.c_void_p, C.c_int32]),
        "gtqa_pool_profile_stages": (C.c_int, [C.c_void_p, C.c_uint32]),
        "gtqa_pool_profile_sample": (C.c_int, [C.c_void_p, C.c_int32]),
        "gtqa_pool_bp_totals": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64)]),
        "gtqa_vidal_residual": (C.c_int, [C.c_void_p, P(C.c_double)]),
        "gtqa_pool_residual": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_int32, P(C.c_double)]),
        "gtqa_set_tuning": (C.c_int, [C.c_int32, C.c_int32]),
        "gtqa_set_bipartition": (C.c_int, [C.c_void_p, P(C.c_uint8)]),
        "gtqa_entropy": (C.c_int, [C.c_void_p, P(C.c_double)]),
        "gtqa_spectral_bipartition": (C.c_int, [C.c_int32, C.c_int32, P(C.c_int32), P(C.c_uint8), P(C.c_int32)]),
        "gtqa_pool_set_bipartition": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_uint8)]),
        "gtqa_pool_entropy": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double)]),
        "gtqa_sample": (C.c_int, [C.c_void_p, P(C.c_double), C.c_double, C.c_int32, P(C.c_int8),
                                  P(C.c_double), P(C.c_double), P(C.c_int32)]),
        "gtqa_pool_sample": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_int32, P(C.c_double), C.c_double,
                                       C.c_int32, P(C.c_int8), P(C.c_double), P(C.c_double), P(C.c_int32)]),
        "gtqa_get_tuning": (C.c_int, [C.c_int32, P(C.c_int32)]),
        "gtqa_x_layer": (C.c_int, [C.c_void_p, C.c_double]),
        "gtqa_pool_x_layer": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_int32, P(C.c_double)]),
        "gtqa_pool_profile_read": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_double),
                                             P(C.c_int64)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    apply_tuning()
    return lib


def set_tuning(knob: str, value: int) -> None:
    _check(load_library().gtqa_set_tuning(TUNE_KNOBS[knob], int(value)), "gtqa_set_tuning")


def get_tuning() -> dict:
    lib = load_library()
    out = {}
    for name, k in TUNE_KNOBS.items():
        v = C.c_int32()
        _check(lib.gtqa_get_tuning(k, C.byref(v)), "gtqa_get_tuning")
        out[name] = int(v.value)
    return out


def apply_tuning(path: str = TUNING_FILE) -> dict | None:
    """Apply the launch configuration the autotuner chose (if its table
    exists); returns the applied knobs."""
    import json
    if _lib is None or not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh)
    knobs = table.get("choice", {})
    for name, value in knobs.items():
        if name in TUNE_KNOBS:
            _check(_lib.gtqa_set_tuning(TUNE_KNOBS[name], int(value)), "gtqa_set_tuning")
    return knobs


class GtqaError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load_library().gtqa_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def _check(code: int, where: str) -> int:
    if code < 0:
        raise GtqaError(code, where)
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


# ---------------------------------------------------------------- ABI mirrors

def gtqa_colour_edges(n: int, edges: np.ndarray) -> np.ndarray:
    lib = load_library()
    e = np.ascontiguousarray(edges, dtype=np.int32)
    out = np.zeros(e.shape[0], dtype=np.uint8)
    _check(lib.gtqa_colour_edges(n, e.shape[0], _ptr(e, C.c_int32), _ptr(out, C.c_uint8)),
           "gtqa_colour_edges")
    return out


def spectral_bipartition(n: int, edges: np.ndarray):
    """(side[n] uint8, cut edges): the library's spectral bipartition (host only)."""
    lib = load_library()
    e = np.ascontiguousarray(edges, dtype=np.int32)
    side = np.zeros(n, dtype=np.uint8)
    cut = C.c_int32()
    _check(lib.gtqa_spectral_bipartition(n, e.shape[0], _ptr(e, C.c_int32), _ptr(side, C.c_uint8),
                                         C.byref(cut)), "gtqa_spectral_bipartition")
    return side, int(cut.value)


def gtqa_footprint_bytes(n: int, n_edges: int, chi: int, precision: int) -> int:
    return int(load_library().gtqa_footprint_bytes(n, n_edges, chi, precision))


def gtqa_version() -> str:
    return load_library().gtqa_version().decode()


def bond_svd(chi: int, cores, svd_rel_cutoff: float = 1e-12, noalloc: bool = False):
    """gtqa_bond_svd (or gtqa_bond_svd_noalloc): the simple update's bond SVD
    on given 2chi x 2chi complex cores [count][2chi][2chi]; returns (column
    norms at exit, descending [count][2chi], Jacobi sweeps [count])."""
    c = np.ascontiguousarray(cores, dtype=np.complex128)
    n2 = 2 * chi
    if c.ndim != 3 or c.shape[1:] != (n2, n2):
        raise ValueError(f"cores must be [count][{n2}][{n2}]")
    flat = np.ascontiguousarray(c.view(np.float64))
    sig = np.zeros((c.shape[0], n2))
    sw = np.zeros(c.shape[0], dtype=np.int32)
    lib = load_library()
    fn = lib.gtqa_bond_svd_noalloc if noalloc else lib.gtqa_bond_svd
    _check(fn(chi, c.shape[0], _ptr(flat, C.c_double), float(svd_rel_cutoff), _ptr(sig, C.c_double),
              _ptr(sw, C.c_int32)), "gtqa_bond_svd_noalloc" if noalloc else "gtqa_bond_svd")
    return sig, sw


def bond_svd_noalloc_max(chi: int) -> int:
    """Largest core count gtqa_bond_svd_noalloc accepts at this chi."""
    return int(load_library().gtqa_bond_svd_noalloc_max(chi))


class _Instance:
    """Keeps the numpy buffers of a gtqa_instance alive."""

    def __init__(self, inst, colour=None):
        self.edges = np.ascontiguousarray(inst.edges, dtype=np.int32)
        self.J = np.ascontiguousarray(inst.J, dtype=np.float64)
        self.h = np.ascontiguousarray(inst.h, dtype=np.float64)
        self.colour = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
        self.c = gtqa_instance(int(inst.n), int(self.edges.shape[0]), _ptr(self.edges, C.c_int32),
                               _ptr(self.J, C.c_double), _ptr(self.h, C.c_double),
                               _ptr(self.colour, C.c_uint8) if self.colour is not None else None)


class TorchDevice:
    """HIP stream and caching-allocator hooks taken from PyTorch.

    By default the library gets a stream of its own (default priority), so
    its launch sequences can be captured as HIP graphs; stream="current"
    uses PyTorch's current stream instead."""

    def __init__(self, stream="own"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch")
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = torch.cuda.Stream() if stream == "own" else torch.cuda.current_stream()
        torch_mod = torch

        def _alloc(nbytes, ctx):
            try:
                return torch_mod.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception as exc:            # reported, then seen by the library as NULL
                import sys
                print(f"gtqa: device allocation of {int(nbytes)} bytes failed: {exc!r}", file=sys.stderr)
                return None

        def _free(ptr, ctx):
            torch_mod.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.allocator = gtqa_allocator(self._alloc_cb, self._free_cb, None)

    @property
    def stream_ptr(self) -> int:
        return int(self.stream.cuda_stream)


def make_options(chi=4, precision="fp64", bp_tol=None, bp_max_sweeps=50, svd_rel_cutoff=1e-12,
                 eig_rel_cutoff=1e-14, regauge="colour", residual_max=1e-3, launch="direct",
                 bp_schedule="colour", device: TorchDevice | None = None):
    lib = load_library()
    o = gtqa_options()
    lib.gtqa_default_options(C.byref(o))
    o.chi = chi
    o.precision = GTQA_MIXED if precision == "mixed" else GTQA_FP64
    if bp_tol is None:
        bp_tol = 1e-6 if precision == "mixed" else 1e-10
    o.bp_tol = bp_tol
    o.bp_max_sweeps = bp_max_sweeps
    o.svd_rel_cutoff = svd_rel_cutoff
    o.eig_rel_cutoff = eig_rel_cutoff
    o.regauge_policy = REGAUGE[regauge]
    o.residual_max = residual_max
    o.launch_mode = LAUNCH[launch]
    o.bp_schedule = BP_SCHEDULE[bp_schedule]
    if device is not None:
        o.stream = device.stream_ptr
        o.allocator = C.pointer(device.allocator)
    return o


def _stats_dict(s: gtqa_step_stats):
    k = min(int(s.n_regauges), 8)
    return {"n_regauges": int(s.n_regauges), "bp_sweeps": [int(s.bp_sweeps[i]) for i in range(k)],
            "bp_dist": [float(s.bp_dist[i]) for i in range(k)], "n_colours": int(s.n_colours),
            "log_fidelity": float(s.log_fidelity), "max_trunc_error": float(s.max_trunc_error),
            "log_fidelity_total": float(s.log_fidelity_total),
            "residual": [float(s.residual[i]) for i in range(min(int(s.n_colours), 8))],
            "entropy": float(s.entropy)}


class TrotterState:
    """One instance: gtqa_init_state / gtqa_trotter_step / gtqa_bp_converge /
    gtqa_readout / gtqa_free_state."""

    def __init__(self, inst, colour=None, device: TorchDevice | None = None, **opts):
        self.lib = load_library()
        self.device = device
        self.opts = make_options(device=device, **opts)
        self._inst = _Instance(inst, colour)
        self.n = int(inst.n)
        h = C.c_void_p()
        _check(self.lib.gtqa_init_state(C.byref(self._inst.c), C.byref(self.opts), C.byref(h)),
               "gtqa_init_state")
        self.handle = h

    def step(self, theta_z: float, theta_x: float, stats: bool = False):
        st = gtqa_step_stats() if stats else None
        rc = _check(self.lib.gtqa_trotter_step(self.handle, float(theta_z), float(theta_x),
                                               C.byref(st) if st is not None else None),
                    "gtqa_trotter_step")
        return (rc, _stats_dict(st)) if stats else rc

    def x_layer(self, theta_x: float):
        """The mixing layer alone (gtqa_x_layer)."""
        return _check(self.lib.gtqa_x_layer(self.handle, float(theta_x)), "gtqa_x_layer")

    def bp_converge(self, tol: float, max_sweeps: int, regauge: bool = False, random_seed=None):
        """gtqa_bp_converge: warm start, or Alg. 1's random start from
        SplitMix64(random_seed) when random_seed is given."""
        sw = C.c_int32()
        dist = C.c_double()
        flags = (GTQA_BP_REGAUGE if regauge else 0) | (GTQA_BP_RANDOM if random_seed is not None else 0)
        seed = 0 if random_seed is None else int(random_seed) & ((1 << 64) - 1)
        rc = _check(self.lib.gtqa_bp_converge(self.handle, tol, max_sweeps, flags, seed,
                                              C.byref(sw), C.byref(dist)), "gtqa_bp_converge")
        return rc, int(sw.value), float(dist.value)

    def set_network(self, gamma, lam):
        """gtqa_set_network: gamma [n][2][chi][chi][chi] complex, lam [E][chi]."""
        g = np.ascontiguousarray(gamma, dtype=np.complex128)
        lm = np.ascontiguousarray(lam, dtype=np.float64)
        chi = self.opts.chi
        if g.shape != (self.n, 2, chi, chi, chi) or lm.shape != (self._inst.edges.shape[0], chi):
            raise ValueError("network shapes do not match the instance and chi")
        gf = np.ascontiguousarray(g.view(np.float64))
        return _check(self.lib.gtqa_set_network(self.handle, _ptr(gf, C.c_double), _ptr(lm, C.c_double)),
                      "gtqa_set_network")

    def get_network(self):
        """gtqa_get_network: (gamma [n][2][chi][chi][chi] complex, lam [E][chi])."""
        chi = self.opts.chi
        gf = np.zeros((self.n, 2, chi, chi, chi, 2))
        lm = np.zeros((self._inst.edges.shape[0], chi))
        _check(self.lib.gtqa_get_network(self.handle, _ptr(gf, C.c_double), _ptr(lm, C.c_double)),
               "gtqa_get_network")
        return gf[..., 0] + 1j * gf[..., 1], lm

    def sample(self, u, tol: float, max_sweeps: int):
        """BP-guided measurement sampling (gtqa_sample): x, E(x), outcome
        probabilities and BP sweeps per qubit."""
        uu = np.ascontiguousarray(u, dtype=np.float64)
        if uu.size != self.n:
            raise ValueError("u needs one entry per vertex")
        x = np.zeros(self.n, dtype=np.int8)
        E = np.zeros(1)
        prob = np.zeros(self.n)
        sw = np.zeros(self.n, dtype=np.int32)
        rc = _check(self.lib.gtqa_sample(self.handle, _ptr(uu, C.c_double), float(tol), int(max_sweeps),
                                         _ptr(x, C.c_int8), _ptr(E, C.c_double), _ptr(prob, C.c_double),
                                         _ptr(sw, C.c_int32)), "gtqa_sample")
        return {"x": x, "energy": float(E[0]), "prob": prob, "sweeps": sw, "rc": rc}

    def set_bipartition(self, side):
        sd = np.ascontiguousarray(side, dtype=np.uint8)
        if sd.size != self.n:
            raise ValueError("side needs one entry per vertex")
        _check(self.lib.gtqa_set_bipartition(self.handle, _ptr(sd, C.c_uint8)), "gtqa_set_bipartition")

    def entropy(self) -> float:
        """S* over the bipartition (gtqa_entropy)."""
        v = C.c_double()
        _check(self.lib.gtqa_entropy(self.handle, C.byref(v)), "gtqa_entropy")
        return float(v.value)

    def vidal_residual(self) -> float:
        """R of App. C for the current network (gtqa_vidal_residual)."""
        r = C.c_double()
        _check(self.lib.gtqa_vidal_residual(self.handle, C.byref(r)), "gtqa_vidal_residual")
        return float(r.value)

    def readout(self, from_messages: bool = False):
        z = np.zeros(self.n)
        rho = np.zeros((self.n, 2, 2, 2))
        x = np.zeros(self.n, dtype=np.int8)
        E = np.zeros(1)
        rc = _check(self.lib.gtqa_readout(self.handle,
                                          GTQA_READ_FROM_MESSAGES if from_messages else GTQA_READ_FROM_VIDAL,
                                          _ptr(z, C.c_double), _ptr(rho, C.c_double),
                                          _ptr(x, C.c_int8), _ptr(E, C.c_double)), "gtqa_readout")
        return {"z": z, "rho": rho[..., 0] + 1j * rho[..., 1], "x": x, "energy": float(E[0]), "rc": rc}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gtqa_free_state(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Many resident instances of one chi/precision: gtqa_pool_*."""

    def __init__(self, chi=4, precision="fp64", max_vertices=1 << 16, max_edges=None, max_slots=64,
                 budget_bytes=0, device: TorchDevice | None = None, **opts):
        self.lib = load_library()
        self.device = device
        po = gtqa_pool_options()
        po.base = make_options(chi=chi, precision=precision, device=device, **opts)
        po.max_vertices = int(max_vertices)
        po.max_edges = int(max_edges if max_edges is not None else (3 * max_vertices) // 2)
        po.max_slots = int(max_slots)
        po.budget_bytes = int(budget_bytes)
        self._po = po
        h = C.c_void_p()
        _check(self.lib.gtqa_pool_create(C.byref(po), C.byref(h)), "gtqa_pool_create")
        self.handle = h
        self._inst = {}
        self.n = {}

    def admit(self, inst, colour=None) -> int:
        ci = _Instance(inst, colour)
        slot = C.c_int32(-1)
        rc = self.lib.gtqa_pool_admit(self.handle, C.byref(ci.c), C.byref(slot))
        if rc == GTQA_BUSY:
            return -1
        _check(rc, "gtqa_pool_admit")
        self._inst[slot.value] = ci
        self.n[slot.value] = int(inst.n)
        return int(slot.value)

    def step(self, slots, theta_z, theta_x, stats: bool = False):
        s = np.ascontiguousarray(slots, dtype=np.int32)
        tz = np.ascontiguousarray(np.broadcast_to(theta_z, s.shape), dtype=np.float64)
        tx = np.ascontiguousarray(np.broadcast_to(theta_x, s.shape), dtype=np.float64)
        st = (gtqa_step_stats * s.size)() if stats else None
        rc = _check(self.lib.gtqa_pool_step(self.handle, _ptr(s, C.c_int32), _ptr(tz, C.c_double),
                                            _ptr(tx, C.c_double), s.size, st), "gtqa_pool_step")
        return (rc, [_stats_dict(x) for x in st]) if stats else rc

    def readout(self, slot: int):
        n = self.n[slot]
        z = np.zeros(n)
        rho = np.zeros((n, 2, 2, 2))
        x = np.zeros(n, dtype=np.int8)
        E = np.zeros(1)
        rc = _check(self.lib.gtqa_pool_readout(self.handle, slot, _ptr(z, C.c_double),
                                               _ptr(rho, C.c_double), _ptr(x, C.c_int8),
                                               _ptr(E, C.c_double)), "gtqa_pool_readout")
        return {"z": z, "rho": rho[..., 0] + 1j * rho[..., 1], "x": x, "energy": float(E[0]), "rc": rc}

    def release(self, slot: int):
        _check(self.lib.gtqa_pool_release(self.handle, slot), "gtqa_pool_release")
        self._inst.pop(slot, None)
        self.n.pop(slot, None)

    def sample(self, slots, u, tol: float, max_sweeps: int):
        """gtqa_pool_sample: per slot (x, E(x), prob, sweeps), u concatenated in slot order."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        ns = [self.n[int(k)] for k in s]
        tot = sum(ns)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        if uu.size != tot:
            raise ValueError("u needs one entry per vertex of every slot")
        x = np.zeros(tot, dtype=np.int8)
        E = np.zeros(s.size)
        prob = np.zeros(tot)
        sw = np.zeros(tot, dtype=np.int32)
        _check(self.lib.gtqa_pool_sample(self.handle, _ptr(s, C.c_int32), s.size, _ptr(uu, C.c_double),
                                         float(tol), int(max_sweeps), _ptr(x, C.c_int8), _ptr(E, C.c_double),
                                         _ptr(prob, C.c_double), _ptr(sw, C.c_int32)), "gtqa_pool_sample")
        out, o = [], 0
        for i, n in enumerate(ns):
            out.append({"x": x[o:o + n], "energy": float(E[i]), "prob": prob[o:o + n], "sweeps": sw[o:o + n]})
            o += n
        return out

    def set_bipartition(self, slot: int, side):
        sd = np.ascontiguousarray(side, dtype=np.uint8)
        if sd.size != self.n[slot]:
            raise ValueError("side needs one entry per vertex")
        _check(self.lib.gtqa_pool_set_bipartition(self.handle, slot, _ptr(sd, C.c_uint8)),
               "gtqa_pool_set_bipartition")

    def entropy(self, slot: int) -> float:
        v = C.c_double()
        _check(self.lib.gtqa_pool_entropy(self.handle, slot, C.byref(v)), "gtqa_pool_entropy")
        return float(v.value)

    def x_layer(self, slots, theta_x):
        """The mixing layer alone on each listed slot (gtqa_pool_x_layer);
        theta_x: one angle per slot or a scalar."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        th = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_x, dtype=np.float64), s.shape))
        return _check(self.lib.gtqa_pool_x_layer(self.handle, _ptr(s, C.c_int32), s.size, _ptr(th, C.c_double)),
                      "gtqa_pool_x_layer")

    def residual(self, slots):
        """R of App. C for each listed slot (gtqa_pool_residual)."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        out = np.zeros(s.size)
        _check(self.lib.gtqa_pool_residual(self.handle, _ptr(s, C.c_int32), s.size, _ptr(out, C.c_double)),
               "gtqa_pool_residual")
        return out

    def free_bytes(self) -> int:
        return int(self.lib.gtqa_pool_free_bytes(self.handle))

    def set_bp(self, tol: float, max_sweeps: int):
        """gtqa_pool_set_bp: the BP stop rule of later steps."""
        _check(self.lib.gtqa_pool_set_bp(self.handle, float(tol), int(max_sweeps)), "gtqa_pool_set_bp")

    def set_network(self, slot: int, gamma, lam):
        """gtqa_pool_set_network for one slot."""
        g = np.ascontiguousarray(gamma, dtype=np.complex128)
        lm = np.ascontiguousarray(lam, dtype=np.float64)
        gf = np.ascontiguousarray(g.view(np.float64))
        _check(self.lib.gtqa_pool_set_network(self.handle, slot, _ptr(gf, C.c_double), _ptr(lm, C.c_double)),
               "gtqa_pool_set_network")

    def bp_totals(self, slot: int):
        """(BP sweeps, re-gaugings) of a slot since its admission."""
        sw = C.c_int64()
        rg = C.c_int64()
        _check(self.lib.gtqa_pool_bp_totals(self.handle, slot, C.byref(sw), C.byref(rg)), "gtqa_pool_bp_totals")
        return int(sw.value), int(rg.value)

    def profile(self, enable: bool):
        _check(self.lib.gtqa_pool_profile(self.handle, 1 if enable else 0), "gtqa_pool_profile")

    def profile_stages(self, stages):
        """Time only the named stages (names of STAGES)."""
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
        _check(self.lib.gtqa_pool_profile_stages(self.handle, mask), "gtqa_pool_profile_stages")

    def profile_sample(self, every: int):
        """Time the launches of one pool step in every `every`."""
        _check(self.lib.gtqa_pool_profile_sample(self.handle, int(every)), "gtqa_pool_profile_sample")

    def profile_read(self):
        """{stage: (launches, total_ms, items)} of the launches timed since enabling."""
        out = {}
        for i, name in enumerate(STAGES):
            n = C.c_int64()
            ms = C.c_double()
            it = C.c_int64()
            _check(self.lib.gtqa_pool_profile_read(self.handle, i, C.byref(n), C.byref(ms), C.byref(it)),
                   "gtqa_pool_profile_read")
            out[name] = (int(n.value), float(ms.value), int(it.value))
        return out

    def resident(self) -> int:
        return int(self.lib.gtqa_pool_resident(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gtqa_pool_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
