"""MI355X-native Kruskal-Wallis SNP x trait scan (kruX, arXiv:1307.3519).

The compute lives in the HIP library ``libkrux.so`` (C ABI declared in
``include/krux.h``); ``paper_1307_3519_amd.krux`` is its thin ctypes binding.
The binding is imported on first use so that the input generators in
``paper_1307_3519_amd.datagen`` can be used without a GPU.
"""
import importlib


def __getattr__(name):
    if name in ("krux", "datagen", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
