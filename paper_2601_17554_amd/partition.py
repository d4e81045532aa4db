"""Host-side partitioning of events for partitioned attention (the paper's closing remark in
Sec. 5.3 on partitioning the event before the correlation-building layers, and the block attention
of Sec. 9).

An event's valid elements are cut into cells of the (eta, phi) plane of about ``target`` elements
each: K = ceil(N / target) cells, ceil(sqrt(K)) bands of equal element count along eta, each band
cut into equal-count ranges of phi. The rows of every event are reordered so that each cell is a
contiguous row range, and the cells become the attention partitions of the library's batch
description (mlpf_batch_t.attn_parts): an element then attends only to the elements of its own
cell. Which feature columns hold eta and phi is the caller's; the synthetic inputs of this
repository carry no detector geometry, and their columns 6, 7 and 8 stand in for eta, sin phi and
cos phi.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

ETA_COL, SIN_COL, COS_COL = 6, 7, 8


def cells(eta: np.ndarray, phi: np.ndarray, target: int) -> Tuple[np.ndarray, np.ndarray]:
    """(order, sizes) of one event's elements: ``order`` lists the element indices cell by cell,
    ``sizes`` the cell sizes (all > 0, summing to len(eta))."""
    n = len(eta)
    if n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    k = max(1, math.ceil(n / max(1, target)))
    bands = max(1, math.ceil(math.sqrt(k)))
    per_band = max(1, math.ceil(k / bands))
    by_eta = np.argsort(eta, kind="stable")
    order, sizes = [], []
    for band in np.array_split(by_eta, bands):
        if band.size == 0:
            continue
        band = band[np.argsort(phi[band], kind="stable")]
        for cell in np.array_split(band, per_band):
            if cell.size:
                order.append(cell)
                sizes.append(cell.size)
    return np.concatenate(order), np.asarray(sizes, np.int64)


def partition_batch(x: np.ndarray, row_start: np.ndarray, n_valid, target: int = 512,
                    eta_col: int = ETA_COL, sin_col: int = SIN_COL, cos_col: int = COS_COL):
    """Partitions every event of a packed batch (x [T][F], row_start [E+1], n_valid [E] or None).

    Returns (perm, part_row_start, part_n_valid): ``perm`` [T] is the row order that makes every
    cell a contiguous row range (x[perm] is the reordered batch; rows that are not valid elements
    keep their place); cell p is rows part_row_start[p] .. part_row_start[p] + part_n_valid[p] - 1
    of the reordered batch, and part_row_start[p + 1] is the next cell's first row, or, for the
    last cell of an event, the next event's first row (so the event's padding rows are in its
    last cell's span but not among its valid rows). These are the row_start and n_valid of the
    library's attention partitions. Outputs of the reordered batch go back to the original row
    order with out[np.argsort(perm)]."""
    row_start = np.asarray(row_start, np.int64)
    t = int(row_start[-1]) if len(row_start) else 0
    perm = np.arange(t, dtype=np.int64)
    starts, counts = [], []
    for e in range(len(row_start) - 1):
        s = int(row_start[e])
        nv = int(row_start[e + 1] - s) if n_valid is None else int(n_valid[e])
        if nv == 0:
            continue
        xe = x[s:s + nv]
        order, sizes = cells(xe[:, eta_col], np.arctan2(xe[:, sin_col], xe[:, cos_col]), target)
        perm[s:s + nv] = s + order
        offs = s + np.concatenate([[0], np.cumsum(sizes)[:-1]])
        starts.extend(offs.tolist())
        counts.extend(sizes.tolist())
    starts.append(t)
    return perm, np.asarray(starts, np.int32), np.asarray(counts, np.int32)
