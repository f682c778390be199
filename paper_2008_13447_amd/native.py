"""ctypes binding of the VALMOD C ABI (include/valmod.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libvalmod.so``. The functions keep the C names (``valmod_plan``,
``valmod_run``, ...); ``run_valmod`` is a convenience wrapper that allocates the
workspace and outputs as torch device tensors and calls them.

The library must have been built (``__graft_entry__.build()``); importing
this module does not build it, and a missing library raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Union

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvalmod.so")

VALMOD_OK = 0
STATUS = {0: "VALMOD_OK", -1: "VALMOD_E_ARG", -2: "VALMOD_E_TOO_SHORT", -3: "VALMOD_E_NOMEM",
          -4: "VALMOD_E_HIP", -5: "VALMOD_E_LAYOUT", -6: "VALMOD_E_DEVICE", -7: "VALMOD_E_SCRATCH"}
DTYPE = {"f32": 0, "f64": 1}
PRECISION = {"fp64": 0, "fp32": 1}
MODE = {"exact": 0, "paper": 1}
PATH = {"auto": 0, "full": 1, "recompute": 2}
NSTATS = 15
STAT_NAMES = ["valid", "failed", "recomputed", "full_pass", "flat", "appends", "pass_events", "pass_hits",
              "fp64_items", "passes", "partial", "mth_certified", "mth_recomputed", "mth_pruned", "overflowed"]

# (name, C type) of every function declared in include/valmod.h
EXPORTS = ["valmod_plan", "valmod_workspace_bytes", "valmod_output_sizes", "valmod_series_layout",
           "valmod_run", "valmod_run_noalloc", "valmod_run_status", "valmod_autotune", "valmod_plan_free", "valmod_status_str",
           "valmod_last_pass_timing", "valmod_rounding_bound"]


class ValmodConfig(ctypes.Structure):
    _fields_ = [
        ("num_series", ctypes.c_int32),
        ("n", ctypes.POINTER(ctypes.c_int64)),
        ("l_min", ctypes.POINTER(ctypes.c_int32)),
        ("l_max", ctypes.POINTER(ctypes.c_int32)),
        ("p", ctypes.c_int32),
        ("k_motifs", ctypes.c_int32),
        ("k_discords", ctypes.c_int32),
        ("excl_den", ctypes.c_int32),
        ("flat_eps", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("refresh_R", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("m_discords", ctypes.c_int32),
        ("mset_radius", ctypes.c_double),
        ("mset_cap", ctypes.c_int32),
    ]


OUTPUT_FIELDS = ["prof_dist", "prof_idx", "valmp_norm", "valmp_dist", "valmp_len", "valmp_idx",
                 "motif_ab", "motif_d", "discord_on", "discord_d", "g_motif_abl", "g_motif_d",
                 "g_discord_onl", "g_discord_d", "stats", "mdiscord_on", "mdiscord_d", "g_mdiscord_onl",
                 "g_mdiscord_d", "mset_count", "mset_off", "mset_dist"]


class ValmodOutputs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in OUTPUT_FIELDS]


class ValmodSizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ["prof", "valmp", "motif", "discord", "g_motif", "g_discord", "stats", "series", "mdiscord",
                 "g_mdiscord", "mset"]]


class ValmodLayout(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ["series", "prof", "valmp", "motif", "discord", "g_motif", "g_discord", "stats",
                 "n", "n0", "nlen"]] + [("l_min", ctypes.c_int32), ("l_max", ctypes.c_int32)] + \
        [("mdiscord", ctypes.c_int64), ("g_mdiscord", ctypes.c_int64), ("mset", ctypes.c_int64)]


_lib = None


class ValmodError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status_str(status)})")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libvalmod.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.valmod_plan.argtypes = [ctypes.POINTER(ValmodConfig), ctypes.POINTER(P)]
    L.valmod_plan.restype = ctypes.c_int
    L.valmod_workspace_bytes.argtypes = [P]
    L.valmod_workspace_bytes.restype = ctypes.c_size_t
    L.valmod_output_sizes.argtypes = [P, ctypes.POINTER(ValmodSizes)]
    L.valmod_output_sizes.restype = ctypes.c_int
    L.valmod_series_layout.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ValmodLayout)]
    L.valmod_series_layout.restype = ctypes.c_int
    L.valmod_run.argtypes = [P, P, P, ctypes.POINTER(ValmodOutputs), P]
    L.valmod_run.restype = ctypes.c_int
    L.valmod_run_noalloc.argtypes = [P, P, ctypes.POINTER(ValmodOutputs), P]
    L.valmod_run_noalloc.restype = ctypes.c_int
    L.valmod_run_status.argtypes = [P, P]
    L.valmod_run_status.restype = ctypes.c_int
    L.valmod_rounding_bound.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double]
    L.valmod_rounding_bound.restype = ctypes.c_double
    L.valmod_autotune.argtypes = [P, P, P, ctypes.POINTER(ValmodOutputs), P, ctypes.POINTER(ctypes.c_int32)]
    L.valmod_autotune.restype = ctypes.c_int
    L.valmod_plan_free.argtypes = [P]
    L.valmod_plan_free.restype = None
    L.valmod_status_str.argtypes = [ctypes.c_int]
    L.valmod_status_str.restype = ctypes.c_char_p
    L.valmod_last_pass_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.valmod_last_pass_timing.restype = ctypes.c_int
    _lib = L
    return L


def status_str(status: int) -> str:
    return lib().valmod_status_str(int(status)).decode()


def _check(rc: int, where: str):
    if rc != VALMOD_OK:
        raise ValmodError(rc, where)


def make_config(n: Sequence[int], l_min: Sequence[int], l_max: Sequence[int], p: int = 0,
                k_motifs: int = 1, k_discords: int = 1, excl_den: int = 4, flat_eps: float = 0.0,
                dtype: str = "f32", precision: str = "fp64", refresh_R: int = 0, path: str = "auto",
                device: int = 0, lanes: int = 0, graph: bool = False, mode: str = "exact",
                m_discords: int = 1, mset_radius: float = 0.0, mset_cap: int = 0):
    """Build a ValmodConfig; returns (config, keepalive arrays)."""
    S = len(n)
    na = (ctypes.c_int64 * S)(*[int(v) for v in n])
    lo = (ctypes.c_int32 * S)(*[int(v) for v in l_min])
    hi = (ctypes.c_int32 * S)(*[int(v) for v in l_max])
    cfg = ValmodConfig(S, ctypes.cast(na, ctypes.POINTER(ctypes.c_int64)),
                       ctypes.cast(lo, ctypes.POINTER(ctypes.c_int32)),
                       ctypes.cast(hi, ctypes.POINTER(ctypes.c_int32)), int(p), int(k_motifs),
                       int(k_discords), int(excl_den), float(flat_eps), DTYPE[dtype], PRECISION[precision],
                       int(refresh_R), PATH[path], int(device), int(lanes), 1 if graph else 0, MODE[mode],
                       int(m_discords), float(mset_radius), int(mset_cap))
    return cfg, (na, lo, hi)


def valmod_plan(cfg: ValmodConfig) -> int:
    """Validate the configuration and return a plan handle (int)."""
    h = ctypes.c_void_p()
    _check(lib().valmod_plan(ctypes.byref(cfg), ctypes.byref(h)), "valmod_plan")
    return h.value


def valmod_plan_status(cfg: ValmodConfig) -> int:
    """Status code of valmod_plan without raising (frees a successful plan)."""
    h = ctypes.c_void_p()
    rc = lib().valmod_plan(ctypes.byref(cfg), ctypes.byref(h))
    if rc == VALMOD_OK:
        lib().valmod_plan_free(h)
    return rc


def valmod_workspace_bytes(plan: int) -> int:
    return int(lib().valmod_workspace_bytes(plan))


def valmod_output_sizes(plan: int) -> Dict[str, int]:
    s = ValmodSizes()
    _check(lib().valmod_output_sizes(plan, ctypes.byref(s)), "valmod_output_sizes")
    return {f: getattr(s, f) for f, _ in ValmodSizes._fields_}


def valmod_series_layout(plan: int, s: int) -> Dict[str, int]:
    out = ValmodLayout()
    _check(lib().valmod_series_layout(plan, s, ctypes.byref(out)), "valmod_series_layout")
    return {f: getattr(out, f) for f, _ in ValmodLayout._fields_}


def valmod_run(plan: int, series_ptr: int, workspace_ptr: int, outputs: ValmodOutputs,
               stream: Optional[int] = None) -> None:
    """Enqueue a run (returns before it completes; see valmod_run_status)."""
    _check(lib().valmod_run(plan, series_ptr, workspace_ptr, ctypes.byref(outputs), stream),
           "valmod_run")


def valmod_run_status(plan: int, stream: Optional[int] = None) -> None:
    """Wait for the plan's last run and raise if it reported an error."""
    _check(lib().valmod_run_status(plan, stream), "valmod_run_status")


def valmod_rounding_bound(precision: str, H: int, L: int, phi: float, psi: float, xi: float) -> float:
    """Rounding bound of the diagonal pass for one work item (host function)."""
    return float(lib().valmod_rounding_bound(PRECISION[precision], int(H), int(L), float(phi), float(psi),
                                             float(xi)))


def valmod_autotune(plan: int, series_ptr: int, workspace_ptr: int, outputs: ValmodOutputs,
                    stream: Optional[int] = None):
    """Returns (segment height, diagonals per lane, p) of the tuned series."""
    chosen = (ctypes.c_int32 * 3)()
    _check(lib().valmod_autotune(plan, series_ptr, workspace_ptr, ctypes.byref(outputs), stream, chosen),
           "valmod_autotune")
    return int(chosen[0]), int(chosen[1]), int(chosen[2])


def valmod_plan_free(plan: int) -> None:
    lib().valmod_plan_free(plan)


def valmod_last_pass_timing(plan: int):
    ms = ctypes.c_double()
    launches = ctypes.c_int64()
    cells = ctypes.c_int64()
    _check(lib().valmod_last_pass_timing(plan, ctypes.byref(ms), ctypes.byref(launches),
                                         ctypes.byref(cells)), "valmod_last_pass_timing")
    return ms.value, launches.value, cells.value


class Valmod:
    """A plan plus its torch-allocated workspace and outputs on one GPU."""

    def __init__(self, series: Union["torch.Tensor", List["torch.Tensor"]], l_min, l_max, p: int = 0,
                 k_motifs: int = 1, k_discords: int = 1, excl_den: int = 4, flat_eps: float = 0.0,
                 precision: str = "fp64", refresh_R: int = 0, path: str = "auto", lanes: int = 0,
                 graph: bool = False, mode: str = "exact", m_discords: int = 1, mset_radius: float = 0.0,
                 mset_cap: int = 0, skip: Sequence[str] = ()):
        """skip: names of outputs passed as NULL (not written by the run)."""
        import torch

        if isinstance(series, torch.Tensor):
            series = [series]
        if not series or any((not s.is_cuda) for s in series):
            raise ValueError("series must be CUDA (HIP) tensors")
        dt = series[0].dtype
        if dt not in (torch.float32, torch.float64) or any(s.dtype != dt for s in series):
            raise ValueError("series must all be float32 or all float64")
        S = len(series)
        lo = list(l_min) if isinstance(l_min, (list, tuple)) else [l_min] * S
        hi = list(l_max) if isinstance(l_max, (list, tuple)) else [l_max] * S
        self.device = series[0].device
        self.torch = torch
        cfg, self._keep = make_config([s.numel() for s in series], lo, hi, p, k_motifs, k_discords,
                                      excl_den, flat_eps, "f32" if dt == torch.float32 else "f64",
                                      precision, refresh_R, path, self.device.index or 0, lanes, graph, mode,
                                      m_discords, mset_radius, mset_cap)
        self.m_discords = max(1, int(m_discords))
        self.mset_cap = int(mset_cap) if mset_radius > 0 else 0
        self.plan = valmod_plan(cfg)
        self.graph = bool(graph)
        self._stream = None
        self.k_motifs, self.k_discords = k_motifs, k_discords
        self.sizes = valmod_output_sizes(self.plan)
        self.layouts = [valmod_series_layout(self.plan, s) for s in range(S)]
        dev = self.device
        self.series = torch.cat([s.reshape(-1) for s in series]).contiguous()
        self.workspace = torch.empty(max(valmod_workspace_bytes(self.plan), 256), dtype=torch.uint8,
                                     device=dev)
        z = self.sizes
        f64, i32 = torch.float64, torch.int32
        self.out = {
            "prof_dist": torch.empty(z["prof"], dtype=f64, device=dev),
            "prof_idx": torch.empty(z["prof"], dtype=i32, device=dev),
            "valmp_norm": torch.empty(z["valmp"], dtype=f64, device=dev),
            "valmp_dist": torch.empty(z["valmp"], dtype=f64, device=dev),
            "valmp_len": torch.empty(z["valmp"], dtype=i32, device=dev),
            "valmp_idx": torch.empty(z["valmp"], dtype=i32, device=dev),
            "motif_ab": torch.empty(2 * z["motif"], dtype=i32, device=dev),
            "motif_d": torch.empty(z["motif"], dtype=f64, device=dev),
            "discord_on": torch.empty(2 * z["discord"], dtype=i32, device=dev),
            "discord_d": torch.empty(z["discord"], dtype=f64, device=dev),
            "g_motif_abl": torch.empty(3 * z["g_motif"], dtype=i32, device=dev),
            "g_motif_d": torch.empty(2 * z["g_motif"], dtype=f64, device=dev),
            "g_discord_onl": torch.empty(3 * z["g_discord"], dtype=i32, device=dev),
            "g_discord_d": torch.empty(2 * z["g_discord"], dtype=f64, device=dev),
            "stats": torch.empty(z["stats"], dtype=torch.int64, device=dev),
            "mdiscord_on": torch.empty(max(1, 2 * z["mdiscord"]), dtype=i32, device=dev),
            "mdiscord_d": torch.empty(max(1, z["mdiscord"]), dtype=f64, device=dev),
            "g_mdiscord_onl": torch.empty(max(1, 3 * z["g_mdiscord"]), dtype=i32, device=dev),
            "g_mdiscord_d": torch.empty(max(1, 2 * z["g_mdiscord"]), dtype=f64, device=dev),
            "mset_count": torch.empty(max(1, z["g_motif"] if z["mset"] else 0), dtype=i32, device=dev),
            "mset_off": torch.empty(max(1, z["mset"]), dtype=i32, device=dev),
            "mset_dist": torch.empty(max(1, z["mset"]), dtype=f64, device=dev),
        }
        bad = set(skip) - set(OUTPUT_FIELDS)
        if bad:
            raise ValueError(f"unknown outputs {sorted(bad)}")
        self.skip = set(skip)
        for f in self.skip:
            self.out[f] = None
        self._outs = ValmodOutputs(*[None if self.out[f] is None else self.out[f].data_ptr()
                                     for f in OUTPUT_FIELDS])

    def _stream_for(self, stream):
        torch = self.torch
        if stream is None and self.graph:
            # graph capture needs a stream other than the legacy default one
            if self._stream is None:
                self._stream = torch.cuda.Stream(self.device)
            stream = self._stream
        return stream if stream is not None else torch.cuda.current_stream(self.device)

    def run(self, stream=None, sync: bool = True) -> None:
        """Enqueue one run; with sync (default) also wait for it and check its status."""
        st = self._stream_for(stream)
        valmod_run(self.plan, self.series.data_ptr(), self.workspace.data_ptr(), self._outs,
                   st.cuda_stream)
        if sync:
            valmod_run_status(self.plan, st.cuda_stream)

    def status(self, stream=None) -> None:
        """Wait for the last enqueued run and raise if it reported an error."""
        valmod_run_status(self.plan, self._stream_for(stream).cuda_stream)

    def autotune(self, stream=None):
        """Empirical pass geometry and p (see valmod_autotune); returns (H, K, p) of the tuned series."""
        st = self._stream_for(stream)
        return valmod_autotune(self.plan, self.series.data_ptr(), self.workspace.data_ptr(), self._outs,
                               st.cuda_stream)

    def pass_timing(self):
        """(ms, launches, cells) of the diagonal-pass kernels of the last run."""
        return valmod_last_pass_timing(self.plan)

    def result(self, s: int = 0) -> Dict[str, np.ndarray]:
        """Host copy of the outputs of series s, reshaped like the oracle's."""
        L = self.layouts[s]
        n0, nl = L["n0"], L["nlen"]
        km, kd = self.k_motifs, self.k_discords
        def sl(key, a, b, shape):  # only the series' slice is copied; a skipped output reads back as None
            t = self.out[key]
            return None if t is None else t[a:b].cpu().numpy().reshape(shape)

        out = dict(
            prof_dist=sl("prof_dist", L["prof"], L["prof"] + nl * n0, (nl, n0)),
            prof_idx=sl("prof_idx", L["prof"], L["prof"] + nl * n0, (nl, n0)),
            valmp_norm=sl("valmp_norm", L["valmp"], L["valmp"] + n0, (n0,)),
            valmp_dist=sl("valmp_dist", L["valmp"], L["valmp"] + n0, (n0,)),
            valmp_len=sl("valmp_len", L["valmp"], L["valmp"] + n0, (n0,)),
            valmp_idx=sl("valmp_idx", L["valmp"], L["valmp"] + n0, (n0,)),
            motif_ab=sl("motif_ab", 2 * L["motif"], 2 * (L["motif"] + nl * km), (nl, km, 2)),
            motif_d=sl("motif_d", L["motif"], L["motif"] + nl * km, (nl, km)),
            discord_on=sl("discord_on", 2 * L["discord"], 2 * (L["discord"] + nl * kd), (nl, kd, 2)),
            discord_d=sl("discord_d", L["discord"], L["discord"] + nl * kd, (nl, kd)),
            g_motif_abl=sl("g_motif_abl", 3 * L["g_motif"], 3 * (L["g_motif"] + km), (km, 3)),
            g_motif_d=sl("g_motif_d", 2 * L["g_motif"], 2 * (L["g_motif"] + km), (km, 2)),
            g_discord_onl=sl("g_discord_onl", 3 * L["g_discord"], 3 * (L["g_discord"] + kd), (kd, 3)),
            g_discord_d=sl("g_discord_d", 2 * L["g_discord"], 2 * (L["g_discord"] + kd), (kd, 2)),
            stats=sl("stats", L["stats"], L["stats"] + nl * NSTATS, (nl, NSTATS)),
        )
        m = self.m_discords
        if m > 1:
            a, g = L["mdiscord"], L["g_mdiscord"]
            out["mdiscord_on"] = sl("mdiscord_on", 2 * a, 2 * (a + nl * m * kd), (nl, m, kd, 2))
            out["mdiscord_d"] = sl("mdiscord_d", a, a + nl * m * kd, (nl, m, kd))
            out["g_mdiscord_onl"] = sl("g_mdiscord_onl", 3 * g, 3 * (g + m * kd), (m, kd, 3))
            out["g_mdiscord_d"] = sl("g_mdiscord_d", 2 * g, 2 * (g + m * kd), (m, kd, 2))
        cap = self.mset_cap
        if cap:
            g, a = L["g_motif"], L["mset"]
            out["mset_count"] = sl("mset_count", g, g + km, (km,))
            out["mset_off"] = sl("mset_off", a, a + km * cap, (km, cap))
            out["mset_dist"] = sl("mset_dist", a, a + km * cap, (km, cap))
        return out

    def close(self):
        if getattr(self, "plan", None):
            valmod_plan_free(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_valmod(x, l_min: int, l_max: int, **kw) -> Dict[str, np.ndarray]:
    """One series through the HIP path; returns host numpy outputs."""
    v = Valmod(x, l_min, l_max, **kw)
    v.run()
    v.torch.cuda.synchronize(v.device)
    out = v.result(0)
    v.close()
    return out
