"""gfx950 (MI355X) implementation of the radiative hot path of arXiv:2511.04277.

The compute lives in ``librad.so`` (hand-written HIP, C ABI in include/rad.h);
this package is its Python binding.  Importing it does not need a GPU; calling
an operation needs the built library and a ROCm device.
"""
from . import _lib
from .api import (Batch, Factors, GebhartREF, absorbed_flux, aggregate_nodes, enforce_lsq, enforce_vf_, gebhart_ref,
                  gebhart_ref_adjoint, node_emissivity, ref_check, steady_temperature, view_fractions)

__all__ = ["Batch", "Factors", "GebhartREF", "absorbed_flux", "aggregate_nodes", "enforce_lsq", "enforce_vf_", "gebhart_ref",
           "gebhart_ref_adjoint", "node_emissivity", "ref_check", "steady_temperature", "view_fractions", "_lib"]
