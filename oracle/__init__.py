"""FP64 CPU oracle for the direct Fourier transform of polygons and closed triangle meshes.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library itself never does, and
this package imports nothing from the library. Everything here is NumPy
float64 / complex128.

What it computes (Maranville, "An implementation of an efficient direct
Fourier transform of polygonal areas and volumes"):

* ``ft2d``  -- F(Q) = area integral of exp(+i Q.r) over a polygon, by the 2D
  divergence theorem (section "Divergence theorem method in 2 dimensions",
  eq. line_integral_generic with its midpoint / sinc form).
* ``ft3d``  -- F(Q) = volume integral of exp(+i Q.r) inside a closed triangle
  mesh, as the sum over faces of eq. single_area_integral with the in-plane
  integral from the 2D result (eq. sum_elements_3d, with the orientation of
  the in-plane edge normal corrected; see ``ft3d``).
* ``ft3d_poly`` -- the same for a closed mesh of planar polygon faces with nu_m
  edges each (eq. sum_elements_3d in its general form).
* ``grad3d`` -- dL/dvertices for a real loss L(F) given dL/dReF + i dL/dImF,
  from the derivative of the same volume integral (transport theorem).
* ``ft3d_dq`` -- grad_Q F(Q) = i times the volume integral of r exp(i Q.r),
  by the divergence theorem with the barycentric face moments of ``grad3d``.
* ``ft3d_regions``, ``grad3d_regions`` -- a density constant on each of
  several closed regions: F = sum_j rho_j F_j, and dL/dv, dL/drho, dL/dQ.
* ``orientation_average`` -- sum_j w_j |F(q s_j)|^2 over a direction
  quadrature (the orientation-averaged scattering intensity).

Removable singularities (Q = 0, Q parallel to a face normal, Q perpendicular
to an edge) are handled by series that follow from the same integrals.

Parity status of every function is stated in its docstring; all are pinned by
the CPU tests (closed forms from the paper, independent exact forms, brute
force quadrature, invariants and finite differences).
"""
from .pft_oracle import (  # noqa: F401
    area2d, volume3d, hsym, simplex_exp_series,
    ft2d, ft2d_edge_terms, ft3d, ft3d_face_terms, face_integrals, ft3d_poly, ft3d_poly_face_terms,
    face_vertex_moments, dft3d_dverts, grad3d, grad3d_vertices, orientation_average,
    ft3d_dq, ft3d_regions, grad3d_regions,
)
