"""Locate and load the in-tree native libraries (fail loudly if they are missing)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str) -> ctypes.CDLL:
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        raise RuntimeError(f"{name} is not built; run `python -m paper_2405_05047_amd.build`")
    return ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
