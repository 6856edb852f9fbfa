"""Shared helpers of the GPU tests (meshes, oracle caches, device checks)."""
import functools
import sys

import numpy as np

import synth
from oracle import efie as oefie
from oracle import rwg


def flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bipyramid():
    """Triangular bipyramid: T = 6, N = 9 (odd order), V = 5."""
    v = np.array([[1, 0, 0], [-0.5, np.sqrt(3) / 2, 0], [-0.5, -np.sqrt(3) / 2, 0], [0, 0, 1.2], [0, 0, -1.1]])
    f = np.array([[0, 1, 3], [1, 2, 3], [2, 0, 3], [1, 0, 4], [2, 1, 4], [0, 2, 4]])
    return v, f


def tetrahedron():
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    return v, f


@functools.lru_cache(maxsize=None)
def icosphere(level):
    return synth.icosphere(level)


@functools.lru_cache(maxsize=None)
def oracle_mesh(level):
    return rwg.build(*icosphere(level))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())
