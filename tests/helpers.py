"""Shared helpers of the tests (no arithmetic of the method)."""

import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zxpar.h")


def header_functions():
    """names of the functions declared in include/zxpar.h"""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:SIM_API\s+)?(?:int|void|const char \*)\s*\*?\s*(sim_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
