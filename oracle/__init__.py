"""Plain FP64 CPU oracle for the radiative hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package; only the tests, the GPU smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP library.

Every function follows the thesis (Frangi, "Novel Numerical Methods for
Accurate Space Thermal Analysis", arXiv:2511.04277) and cites the passage it
implements:

* ``enforce``   - iterative closure + reciprocity enforcer for open systems
                  (Sec. 3.5.5; reciprocity eq. 3.18-3.25, closure eq. 3.36-3.40).
* ``gebhart``   - open-system Gebhart matrix method (Sec. 4.2.3, eq. 4.5;
                  App. B.1-B.2, eq. B.1-B.11) and the REF relations (eq. 4.3-4.4).
* ``adjoint``   - gradients of an objective of B with respect to the per-face
                  emissivity and reflectivity, by the transposed solve.
* ``aggregate`` - multi-node surface relations (Sec. 5.2.3, eq. 5.6-5.7 and
                  eq. 5.28 for one-sided faces).
* ``ahf``       - absorbed heat fluxes from REFs and direct heat fluxes
                  (Sec. 4.2.3, eq. 4.6).
* ``steady``    - radiation-only steady-state node temperatures (Sec. 3.4.4,
                  eq. 3.12-3.14 with GR from REFs, eq. 4.2).
* ``twosided``  - two-sided multi-node relations: node factors, view
                  fractions and node emissivity (eq. 5.17, 5.29, C.4).
* ``lsq``       - least-squares optimum closure + reciprocity enforcer with
                  NNR and SPVA (Sec. 3.5.5, eq. 3.41-3.52; App. A).

All arithmetic is float64.  Functions whose result has a plain definition use
that definition directly (a LAPACK solve, dense products, sums); the iterative
enforcer follows the paper's steps in its order and notation.
"""
from .enforce import closure_step, enforce_vf, reciprocity_step, kappa_fracvar, mae
from .gebhart import form_k_e, gebhart_ref, ref_closure_residual, ref_reciprocity_residual
from .adjoint import gebhart_ref_adjoint
from .aggregate import aggregate_nodes
from .ahf import absorbed_flux
from .steady import steady_temperature
from .twosided import node_emissivity, node_view_factors, view_fractions
from .lsq import enforce_lsq

__all__ = [
    "closure_step", "enforce_vf", "reciprocity_step", "kappa_fracvar", "mae",
    "form_k_e", "gebhart_ref", "ref_closure_residual", "ref_reciprocity_residual",
    "gebhart_ref_adjoint", "aggregate_nodes", "absorbed_flux", "steady_temperature", "node_emissivity", "node_view_factors", "view_fractions", "enforce_lsq",
]
