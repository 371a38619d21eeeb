"""MI355X-native sketched-EI CT operator library (arXiv 2411.05771 hot path).

Submodules load lazily so that importing the seeded input generators
(``paper_2411_05771_amd.synth``) never touches the HIP library.
"""
import importlib

__all__ = ["synth", "capi", "ops", "ei", "batched", "serve", "build", "ttt"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
