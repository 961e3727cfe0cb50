"""Tracker configuration: geometry, field, resolution and cut values.

The defaults here mirror ``tpc_default_config`` of the C library (the
tracker's own defaults); the geometry arrays come from the detector model in
:mod:`synth`.  The values are plain inputs: the test suite hands the same
dict to the HIP tracker and to the FP64 oracle.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import synth


@dataclasses.dataclass
class TrackerConfig:
    row_x: np.ndarray = None
    row_half_y: np.ndarray = None
    bz: float = synth.BZ_TESLA
    sigma_y: float = synth.SIGMA_Y
    sigma_z: float = synth.SIGMA_Z
    grid_hits_per_bin: int = 2
    win_a_y: float = 2.0
    win_b_y: float = 0.5
    win_a_z: float = 2.0
    win_b_z: float = 0.7
    link_nsigma: float = 4.0
    s_max: float = 0.99
    seed_qpt_max: float = 10.0
    c0_sinphi: float = 0.25
    c0_tanl: float = 0.25
    c0_qpt: float = 25.0
    gate_nsigma: float = 3.0
    win_cap: float = 3.0
    edge_margin: float = 1.0
    max_miss: int = 5
    min_tracklet_hits: int = 10
    min_track_hits: int = 10
    min_owned_frac: float = 0.5
    # sector merger (C8): windows on the difference between a segment propagated
    # into the next sector and the segment found there
    merge_dy: float = 2.0
    merge_dz: float = 2.0
    merge_dsinphi: float = 0.05
    merge_dtanl: float = 0.05
    merge_dqpt: float = 1.0

    def __post_init__(self):
        if self.row_x is None or self.row_half_y is None:
            self.row_x, self.row_half_y = synth.row_geometry()

    def as_dict(self):
        return dataclasses.asdict(self)


def default_config(**overrides) -> TrackerConfig:
    return TrackerConfig(**overrides)
