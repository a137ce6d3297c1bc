"""Helpers shared by the GPU parity tests."""
import dataclasses
import sys

import numpy as np


def say(*a):
    """Print-and-flush so a GPU run's log names the case before it runs."""
    print(*a, flush=True)
    sys.stdout.flush()


def f32(a):
    """Round to float32 and back: the values the GPU actually sees."""
    return np.asarray(a, np.float32).astype(np.float64)


def rounded(scene):
    """Copy of a scene with vertices and points rounded to float32, so the
    oracle and the GPU start from identical inputs."""
    s = dataclasses.replace(scene)
    s.verts = f32(scene.verts)
    s.points = f32(scene.points)
    return s


def exact_solution(scene, pts):
    from oracle import field_value
    return np.array([field_value(scene.u_exact, scene.dim, p) for p in pts])


def philox_words(p, j, step, block, seed):
    from oracle import philox4x32_10
    return philox4x32_10([p, j, step, block], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])


def u01(w):
    return (np.asarray(w, np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
