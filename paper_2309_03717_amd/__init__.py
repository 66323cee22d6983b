"""MI355X-native (gfx950 HIP) track x antenna radio-emission library.

For every particle track and every antenna, a straight-line propagator gives
the distance, the effective refractive index and the arrival time, and the
Endpoint electric field or the ZHS vector potential is accumulated into
per-antenna 3-component time traces (the loop of §2 of the paper).

``workloads`` draws seeded synthetic inputs and needs no GPU. The HIP binding
lives in ``radtrace`` and is imported on first use: it raises if the compiled
library is missing rather than falling back to anything else.
"""
import importlib

__all__ = ["workloads", "radtrace"]


def __getattr__(name):
    if name in ("radtrace", "workloads"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
