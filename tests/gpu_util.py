"""Helpers for the GPU tests (marshalling only; no method arithmetic)."""
import sys

import numpy as np

import paper_2601_09477_amd as cmm


def torch():
    import torch as _t
    return _t


def dev(x, dtype=None):
    t = torch()
    a = np.ascontiguousarray(x)
    return t.from_numpy(a).to("cuda", dtype=dtype)


def tables_dev(tab_np):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(tab_np).view(np.int32)).to("cuda")


def host(x):
    return x.detach().cpu().numpy()


def announce(msg):
    """Name the case before any GPU work, flushed (a fault kills the output)."""
    sys.stdout.write(f"[case] {msg}\n")
    sys.stdout.flush()
