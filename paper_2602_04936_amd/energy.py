"""Energy per query from the GPU's own energy accumulator (amd-smi).

The paper reports energy per query for the full scan and for range scans over
prefix buckets (section 6, Theorem "TAL Energy Reduction"; section 7, Table
"TAL range-scan vs full-scan" and the bucket-count figure), sampled from the
board's power telemetry.  Here the socket energy accumulator of the MI355X is
read before and after a sustained run of one path; joules over the run divided
by the queries answered is the energy per query.  The idle draw over the same
length of time is measured too, so the dynamic share can be told apart.

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

    def read_joules(self) -> float:
        try:
            r = self._smi.amdsmi_get_energy_count(self.handle)
        except Exception as e:
            raise EnergyUnavailable(f"amdsmi_get_energy_count failed: {e}") from None
        # accumulator ticks x resolution (microjoules per tick)
        return float(r["energy_accumulator"]) * float(r["counter_resolution"]) * 1e-6

    def measure(self, fn: Callable[[], int], seconds: float, sync_every: int = 8) -> Dict:
        """Call `fn` (which returns the queries it answered) repeatedly for at
        least `seconds` of wall time; return joules, seconds, watts, queries and
        J/query for the run."""
        torch.cuda.synchronize(self.device)
        e0 = self.read_joules()
        t0 = time.perf_counter()
        queries = 0
        calls = 0
        while True:
            queries += int(fn())
            calls += 1
            if calls % sync_every == 0:
                torch.cuda.synchronize(self.device)
                if time.perf_counter() - t0 >= seconds:
                    break
        t1 = time.perf_counter()
        e1 = self.read_joules()
        j = e1 - e0
        dt = t1 - t0
        return {"joules": round(j, 3), "seconds": round(dt, 3), "watts": round(j / dt, 1),
                "queries": queries, "calls": calls,
                "j_per_query": (j / queries) if queries else None}

    def idle_watts(self, seconds: float) -> float:
        torch.cuda.synchronize(self.device)
        e0 = self.read_joules()
        t0 = time.perf_counter()
        time.sleep(seconds)
        e1 = self.read_joules()
        return (e1 - e0) / (time.perf_counter() - t0)

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
