"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This package holds only random-number draws and array shapes.  It contains none of
the method's arithmetic (no keys, no tree, no stencils), so it may be imported by
both sides without coupling them.
"""
from .beam_halo import (beam_halo, batch_specs, uniform_lattice_points, gaussian_blob,
                        paper_beam_3d, BEAM3D, paper_beam_2d, BEAM2D, CONFIGS, BATCH)

__all__ = ["beam_halo", "batch_specs", "uniform_lattice_points", "gaussian_blob", "paper_beam_3d",
           "BEAM3D", "paper_beam_2d", "BEAM2D", "CONFIGS", "BATCH"]
