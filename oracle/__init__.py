"""FP64 CPU oracle for the cell-vertex WENO stabilised residual.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package;
only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code, tables or constants with the HIP
library: bases, quadrature rules, connectivity and every formula are rebuilt
here from the paper's definitions, in float64, in the paper's order.

Modules
-------
basis      Lagrange bases, Gauss / Gauss-Lobatto / Stroud rules (Sec. 2.1).
mesh       vertex patches C(x_i), face neighbours, CG numbering (Sec. 3.2).
geometry   physical derivatives D^k u on affine and bilinear cells.
method     Hermite data, vertex HWENO candidates, cell WENO weights,
           sensor gamma_e (Sec. 3.2, eq. gamma / snorm / pointsnorm),
           shock-capturing quadrature weights alpha_q (Sec. 4),
           stabilised residual and SSP-RK3 (Sec. 2, eq. stabform / sdstab).
learned    a learned replacement of the sensor gamma_e: features of the
           normalised cell and vertex Hermite data, a 48-64-64-1 network,
           its backward pass, Adam (not from the paper; see its docstring).
"""
from .space import Space, build_space
from .method import (hermite_at_vertices, vertex_candidates, cell_sensor, sc_weights,
                     residual, apply_mass_inverse, rk3_step, nodal_interpolate, hweno_limit,
                     positivity_limit, Params)

__all__ = ["Space", "build_space", "hermite_at_vertices", "vertex_candidates", "cell_sensor",
           "sc_weights", "residual", "apply_mass_inverse", "rk3_step", "nodal_interpolate", "hweno_limit",
           "positivity_limit", "Params"]
