"""Energy per hull from the GPU's own energy counter, idle draw subtracted.

The paper reports the energy of its runs from the CPU package's RAPL energy
counters, against the machine at rest (Section 5.7).  The GPU analog used here
reads the device's accumulated-energy counter through the amd-smi library
before and after a loop of hull calls, and subtracts the energy the same GPU
draws when idle for the same time (measured just before, from the same
counter).  Nothing in the hull path depends on this module; when the counter
cannot be read the measurement reports why instead of a number.
"""
from __future__ import annotations

import ctypes
import time


def _hip_bdf(device: int) -> str | None:
    """PCI address of a HIP device ("dddd:bb:dd.f"), or None."""
    try:
        # by soname: the HIP runtime already in the process (torch's), not a second copy
        hip = ctypes.CDLL("libamdhip64.so.7")
        buf = ctypes.create_string_buffer(64)
        if hip.hipDeviceGetPCIBusId(buf, ctypes.c_int(64), ctypes.c_int(device)) != 0:
            return None
        return buf.value.decode().lower()
    except OSError:
        return None


class EnergyCounter:
    """The accumulated-energy counter of one GPU (joules, seconds)."""

    def __init__(self, device: int = 0):
        import amdsmi

        self._smi = amdsmi
        amdsmi.amdsmi_init()
        handles = amdsmi.amdsmi_get_processor_handles()
        if not handles:
            raise RuntimeError("amd-smi sees no GPU")
        want = _hip_bdf(device)
        match = [h for h in handles if want is not None and amdsmi.amdsmi_get_gpu_device_bdf(h).lower() == want]
        if match:
            self.handle = match[0]
        elif len(handles) == 1:
            self.handle = handles[0]  # the only GPU amd-smi sees
        else:
            raise RuntimeError("cannot tell which GPU amd-smi handle is the HIP device")

    def read(self) -> tuple[float, float]:
        e = self._smi.amdsmi_get_energy_count(self.handle)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, e["timestamp"] * 1e-9

    def close(self) -> None:
        try:
            self._smi.amdsmi_shut_down()
        except Exception:
            pass


def measure(step, units_per_step: int, sync, seconds: float = 2.0, idle_seconds: float = 1.0,
            device: int = 0) -> dict:
    """Run step() repeatedly for about `seconds` and return energy figures per
    unit (e.g. per hull): total, and dynamic (idle draw over the same time
    subtracted).  step() enqueues work; sync() waits for it."""
    try:
        ctr = EnergyCounter(device)
    except Exception as e:  # no library, no permission, or no counter
        return {"available": False, "reason": f"{type(e).__name__}: {e}"}
    try:
        sync()
        e0, t0 = ctr.read()
        time.sleep(idle_seconds)
        e1, t1 = ctr.read()
        idle_w = (e1 - e0) / max(t1 - t0, 1e-9)
        step()  # warm
        sync()
        steps = 0
        e0, t0 = ctr.read()
        w0 = time.perf_counter()
        while time.perf_counter() - w0 < seconds:
            step()
            sync()
            steps += 1
        e1, t1 = ctr.read()
        dt = t1 - t0
        total = e1 - e0
        units = steps * units_per_step
        if total <= 0.0 or dt <= 0.0 or units == 0:
            return {"available": False, "reason": "the energy counter did not advance"}
        return {
            "available": True,
            "units": units,
            "seconds": round(dt, 3),
            "idle_w": round(idle_w, 1),
            "load_w": round(total / dt, 1),
            "joules_per_unit": round(total / units, 5),
            "dynamic_joules_per_unit": round(max(total - idle_w * dt, 0.0) / units, 5),
        }
    finally:
        ctr.close()
