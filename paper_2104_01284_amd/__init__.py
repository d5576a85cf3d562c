"""MI355X-native receding-horizon DP eco-driving solver (Zhu et al., ECC 2021).

The solver itself is the HIP library ``libecodp.so`` behind the C ABI in
``include/ecodp.h``; this package holds its ctypes binding (``_lib``), a thin
Python API (``api.Plan``), the autograd wrapper of the adjoint
(``autograd.EcoDPValue``) and the seeded instance generator (``instances``).
Submodules load lazily so that ``instances`` can be used without torch.
"""

__all__ = ["Plan", "EcoDPValue", "instances", "build"]


def __getattr__(name):
    if name == "Plan":
        from .api import Plan
        return Plan
    if name == "EcoDPValue":
        from .autograd import EcoDPValue
        return EcoDPValue
    if name in ("instances", "build", "api", "autograd"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
