"""Helpers for the GPU tests: place host arrays on the device at a chosen
element offset inside a 16-byte line, and compare pairs bitwise."""
import numpy as np
import torch

import paper_1401_0248_amd as tf

DEV = "cuda:0"
TDT = {np.float32: torch.float32, np.float64: torch.float64}


def to_dev(a, shift=0):
    """Device copy of a at `shift` elements past a 256-byte boundary; returns
    (view, misalignment in elements within its 16-byte line)."""
    a = np.ascontiguousarray(a)
    t = torch.empty(a.size + shift + 64, dtype=TDT[a.dtype.type], device=DEV)
    v = t[shift:shift + a.size]
    v.copy_(torch.from_numpy(a))
    mis = (v.data_ptr() % 16) // a.itemsize
    return v, mis


def pair(t):
    """Device (value, error) tensor -> two Python floats (widened exactly)."""
    h = t.detach().cpu().numpy().astype(np.float64)
    return float(h[0]), float(h[1])


def same_bits(a, b):
    """Bitwise equality of two float pairs (as binary64 bit patterns)."""
    A = np.array(a, dtype=np.float64).view(np.uint64)
    B = np.array(b, dtype=np.float64).view(np.uint64)
    return bool(np.all(A == B))


def launch(bt, u, gb, tile=0):
    return tf.Launch(bt, u, gb, 0, tile)
