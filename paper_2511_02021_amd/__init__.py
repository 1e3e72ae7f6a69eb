"""MI355X-native nonhydrostatic dynamical-core substep on the icosahedral
triangular C-grid (velocity tendencies, predictor/corrector horizontal
stencils, column-implicit w/Exner solve) behind the C-ABI library libnhdc.

Submodules are imported lazily: ``inputs`` (grid builder and synthetic case
generator) never loads the HIP library; ``nhdc`` is the binding of libnhdc.
"""
import importlib

__all__ = ["inputs", "nhdc"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
