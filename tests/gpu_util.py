"""Helpers for the GPU tests (device vectors, oracle references, meshes)."""
import numpy as np
import torch

import synthetic as syn


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev())


def rel_l2(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print(msg, flush=True)


MESHES = {
    "sphere512": lambda: syn.sphere(3),
    "sphere2048": lambda: syn.sphere(4),
    "sphere8192": lambda: syn.sphere(5),
    "rbc2048": lambda: syn.rbc(4),
    "ellipsoid2048": lambda: syn.ellipsoid(4, (0.6, 1.3, 1.9)),
    "cells8x512": lambda: syn.rbc_scene(8, 3, 1),
}
