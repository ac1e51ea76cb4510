"""MI355X (gfx950) PRGD tensor-train completion: HIP library + thin binding.

``paper_2501_13385_amd.workloads`` (random draws for synthetic problems) has no
dependency on the compiled library.  The binding ``paper_2501_13385_amd._lib``
loads ``libprgd.so`` on first use and raises if it has not been built.
"""

import importlib

__all__ = ["workloads", "lib", "build"]


def __getattr__(name):
    if name == "lib":
        mod = importlib.import_module(__name__ + "._lib")
        mod.load()
        return mod
    if name in ("workloads", "build", "_lib"):
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
