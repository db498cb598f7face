"""MI355X-native even-odd HISQ Dslash in low-bit storage formats and the
stabilised mixed-precision CG / multi-shift CG solvers around it
("Maximizing the Bang Per Bit", arXiv 2302.09224).

``paper_2302_09224_amd.hisq`` is the Python binding of the C-ABI library
``libhisq.so`` (loaded on first use); ``paper_2302_09224_amd.inputs`` holds the
seeded synthetic inputs.
"""
import importlib

__all__ = ["hisq", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
