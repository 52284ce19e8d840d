"""FP64 CPU oracle for photometric bundle adjustment with proxy templates.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU library is checked against. Only the test suite, the
smoke entry point and the benchmark's CPU-baseline leg may import it; the
product path (the HIP library and its Python binding) never does, and shares
no code, tables or helpers with it.

It follows Ham, Lucey & Singh, "Proxy Templates for Inverse Compositional
Photometric Bundle Adjustment" (arXiv 1704.06967):
  * geometry.py   - warp (eq. 1 / eq:warp), projection and homogeneous
                    coordinates (Notation), the proxy warp phi in its three
                    forms (eq:phi0, eq:phi_grad, eq:phi_update), M and phi*
                    (Sec. 3.4), the IC parameter update (Sec. 3.6, final
                    equations) and the forward-compositional boxplus.
  * image.py      - bilinear image functions (Notation), pyramid, gradients.
  * residuals.py  - per-residual layout, residuals r = I0(x) - If(W(x;p))
                    (Sec. 3.5), Huber weights/energy (eq:energy), FC and IC
                    Jacobian rows (Sec. 3.5, Sec. 3.4).
  * solver.py     - H = J^T W J and g = J^T W r on the absolute parameters,
                    damping + gauge pin, depth Schur complement, Cholesky.
  * gn.py         - the FC and IC-proxy Gauss-Newton loops (Sec. 3.5 steps
                    1-4) over a coarse-to-fine pyramid, convergence test
                    (Sec. 4.1).
  * frontend.py   - the base solution's first steps (Sec. 4.1): Harris
                    corners, robust KLT tracking, geometric bundle adjustment
                    with outlier removal.
  * affine.py     - per-frame affine brightness (log-gain and offset) in the
                    FC iteration, the photometric modelling Sec. 2 names.
Readings of passages where the paper is silent or garbled are listed in the
docstrings where they are applied.
"""
