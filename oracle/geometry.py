"""Disk geometry of the truncated system (paper sec. 4.1 notation, sec. 5 sizes).

Oracle module (test infrastructure only).
"""
from __future__ import annotations

import numpy as np


def mode_offsets(n_modes) -> tuple[np.ndarray, int]:
    """Offsets of each disk's block in the unknown vector.

    Disk p carries modes m = -N_p..N_p (2 N_p + 1 unknowns, sec. 5); blocks are
    concatenated in disk order.  Returns (off[M+1], N_tot)."""
    n = 2 * np.asarray(n_modes, dtype=np.int64) + 1
    off = np.concatenate([[0], np.cumsum(n)])
    return off, int(off[-1])


def pair_geometry(centers) -> tuple[np.ndarray, np.ndarray]:
    """b_pq = |O_p - O_q| and alpha_pq = angle of the vector from O_q to O_p
    (sec. 4.1: the separation vector b_pq is O_q O_p).  Diagonal entries are 0."""
    c = np.asarray(centers, dtype=np.float64)
    dx = c[:, None, 0] - c[None, :, 0]
    dy = c[:, None, 1] - c[None, :, 1]
    return np.hypot(dx, dy), np.arctan2(dy, dx)


def mode_index(n_modes) -> tuple[np.ndarray, np.ndarray]:
    """For every unknown i: its disk p(i) and mode m(i)."""
    disk = np.concatenate([np.full(2 * N + 1, p) for p, N in enumerate(n_modes)])
    m = np.concatenate([np.arange(-N, N + 1) for N in n_modes])
    return disk.astype(np.int64), m.astype(np.int64)
