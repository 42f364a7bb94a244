"""Energy per query from the GPU's own energy accumulator (amd-smi).

The paper reports energy per query for the full scan and for range scans over
prefix buckets (section 6, Theorem "TAL Energy Reduction"; section 7, Table
"TAL range-scan vs full-scan" and the bucket-count figure), sampled from the
board's power telemetry.  Here the socket energy accumulator of the MI355X is
read while one path runs without pause; it advances in coarse steps, so the
power is taken between two of its update edges and divided by the query rate
over the same interval.  The idle draw is measured the same way, so the
dynamic share can be told apart.

amd-smi ships with ROCm as a Python package outside site-packages; when it is
missing, or the driver refuses the query, `EnergyMeter` raises
`EnergyUnavailable` and callers report no energy figure.
"""
from __future__ import annotations

import sys
import time
from typing import Callable, Dict, Optional

import torch

__all__ = ["EnergyMeter", "EnergyUnavailable"]

_AMDSMI_DIRS = ("/opt/rocm/share/amd_smi",)


class EnergyUnavailable(RuntimeError):
    pass


def _import_amdsmi():
    try:
        import amdsmi  # noqa: F401
    except ImportError:
        for d in _AMDSMI_DIRS:
            if d not in sys.path:
                sys.path.append(d)
        try:
            import amdsmi  # noqa: F401
        except Exception as e:  # the package loads its shared library at import
            raise EnergyUnavailable(f"amdsmi not importable: {e}") from None
    import amdsmi
    return amdsmi


def _bdf_of(device: torch.device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{p.pci_domain_id:04x}:{p.pci_bus_id:02x}:{p.pci_device_id:02x}".lower()


def _span(ts0: int, ts1: int, h0: float, h1: float) -> float:
    """Seconds between two accumulator updates: their own timestamps (ns)
    when those agree with the host clock to within a factor of two."""
    host = h1 - h0
    dev = (ts1 - ts0) * 1e-9
    return dev if 0.5 * host <= dev <= 2.0 * host else host


class EnergyMeter:
    """Energy accumulator of the socket that holds `device`."""

    def __init__(self, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = dev
        smi = _import_amdsmi()
        self._smi = smi
        try:
            smi.amdsmi_init(smi.AmdSmiInitFlags.INIT_AMD_GPUS)
        except Exception as e:
            raise EnergyUnavailable(f"amdsmi_init failed: {e}") from None
        try:
            handles = smi.amdsmi_get_processor_handles()
        except Exception as e:
            raise EnergyUnavailable(f"no processor handles: {e}") from None
        want = _bdf_of(dev)
        self.handle = None
        bdfs = []
        for h in handles:
            try:
                b = str(smi.amdsmi_get_gpu_device_bdf(h)).lower()
            except Exception:
                continue
            bdfs.append(b)
            if b.startswith(want):
                self.handle = h
        if self.handle is None and len(handles) == 1:
            self.handle = handles[0]
        if self.handle is None:
            raise EnergyUnavailable(f"device {want} not among amd-smi devices {bdfs}")
        self.read_joules()  # fail here, not in the middle of a measurement

    def _read(self):
        try:
            r = self._smi.amdsmi_get_energy_count(self.handle)
        except Exception as e:
            raise EnergyUnavailable(f"amdsmi_get_energy_count failed: {e}") from None
        # accumulator ticks x resolution (microjoules per tick); timestamp in ns
        return float(r["energy_accumulator"]) * float(r["counter_resolution"]) * 1e-6, int(r["timestamp"])

    def read_joules(self) -> float:
        return self._read()[0]

    def measure(self, fn: Callable[[], int], seconds: float, sync_every: int = 8, max_wait_s: float = 5.0) -> Dict:
        """Run `fn` (which returns the queries it answered) without pause and
        time it between two updates of the energy accumulator at least
        `seconds` apart.  The accumulator advances in coarse steps, so the
        energy is taken between update edges, over the accumulator's own
        timestamps, and the query rate over the host clock between the moments
        the edges were seen.  Returns watts, queries/s and J/query."""
        torch.cuda.synchronize(self.device)
        e_prev, _ = self._read()
        calls = 0
        queries = 0
        edges = []  # (joules, counter timestamp ns, host s, queries done)
        t_begin = time.perf_counter()
        while True:
            queries += int(fn())
            calls += 1
            if calls % sync_every:
                continue
            torch.cuda.synchronize(self.device)
            now = time.perf_counter()
            e, ts = self._read()
            if e != e_prev:
                edges.append((e, ts, now, queries))
                e_prev = e
                if len(edges) >= 2 and now - edges[0][2] >= seconds:
                    break
            if now - t_begin > seconds + max_wait_s:
                break
        if len(edges) < 2:
            return {"error": "the energy accumulator did not advance during the run", "calls": calls}
        (e0, ts0, h0, q0), (e1, ts1, h1, q1) = edges[0], edges[-1]
        span_s = _span(ts0, ts1, h0, h1)
        watts = (e1 - e0) / span_s
        qps = (q1 - q0) / (h1 - h0)
        return {"watts": round(watts, 1), "seconds": round(h1 - h0, 3), "queries_per_s": round(qps, 1),
                "j_per_query": watts / qps if qps > 0 else None, "accumulator_updates": len(edges) - 1}

    def idle_watts(self, seconds: float, max_wait_s: float = 5.0) -> Optional[float]:
        """Average power with the GPU idle, between accumulator updates."""
        torch.cuda.synchronize(self.device)
        e_prev, _ = self._read()
        edges = []
        t_begin = time.perf_counter()
        while time.perf_counter() - t_begin < seconds + max_wait_s:
            time.sleep(0.002)
            e, ts = self._read()
            if e != e_prev:
                edges.append((e, ts, time.perf_counter()))
                e_prev = e
                if len(edges) >= 2 and edges[-1][2] - edges[0][2] >= seconds:
                    break
        if len(edges) < 2:
            return None
        (e0, ts0, h0), (e1, ts1, h1) = edges[0], edges[-1]
        span_s = _span(ts0, ts1, h0, h1)
        return (e1 - e0) / span_s

    def close(self) -> None:
        try:
            self._smi.amdsmi_shut_down()
        except Exception:
            pass


def try_meter(device=None) -> "tuple[Optional[EnergyMeter], Optional[str]]":
    try:
        return EnergyMeter(device), None
    except EnergyUnavailable as e:
        return None, str(e)
