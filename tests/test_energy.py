"""Energy per hull (CPU): the idle draw is subtracted over the same counter
interval, and a missing counter is reported instead of a number."""
import sys
import types

from paper_2510_09417_amd import energy


class _FakeSmi(types.ModuleType):
    """Counter that advances one second and `rate` joules per read."""

    def __init__(self):
        super().__init__("amdsmi")
        self.e = 0.0
        self.t = 0.0
        self.busy = False

    def amdsmi_init(self):
        pass

    def amdsmi_shut_down(self):
        pass

    def amdsmi_get_processor_handles(self):
        return ["gpu0"]

    def amdsmi_get_gpu_device_bdf(self, h):
        return "0000:00:00.0"

    def amdsmi_get_energy_count(self, h):
        self.t += 1.0
        self.e += 300.0 if self.busy else 100.0
        # 15.3 uJ per count, as the real counter; timestamp in ns
        return {"energy_accumulator": int(round(self.e / 15.3e-6)), "counter_resolution": 15.3,
                "timestamp": int(self.t * 1e9)}


def test_idle_subtracted(monkeypatch):
    fake = _FakeSmi()
    monkeypatch.setitem(sys.modules, "amdsmi", fake)

    def step():
        fake.busy = True

    r = energy.measure(step, 2, lambda: None, seconds=0.02, idle_seconds=0.0)
    assert r["available"] and r["idle_w"] == 100.0 and r["load_w"] == 300.0
    assert abs(r["joules_per_unit"] - 300.0 / r["units"]) < 1e-3
    assert abs(r["dynamic_joules_per_unit"] - 200.0 / r["units"]) < 1e-3
    assert r["units"] % 2 == 0


def test_unavailable_counter_is_reported(monkeypatch):
    bad = types.ModuleType("amdsmi")

    def fail():
        raise RuntimeError("no driver")

    bad.amdsmi_init = fail
    monkeypatch.setitem(sys.modules, "amdsmi", bad)
    r = energy.measure(lambda: None, 1, lambda: None, seconds=0.0, idle_seconds=0.0)
    assert r == {"available": False, "reason": "RuntimeError: no driver"}
