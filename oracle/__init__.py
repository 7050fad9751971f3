"""FP64 CPU oracle for the rigid-body Stokes mobility method of Corona, Greengard,
Rachh and Veerapaneni, "An integral equation formulation for rigid bodies in
Stokes flow in three dimensions" (arXiv 1606.07428).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct NumPy
restatement of the discrete method, written from the paper, against which the HIP
path is checked.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path (the C-ABI
library under ``paper_1606_07428_amd``) never imports, links or calls anything
here, and this package imports nothing from the product path.

Modules
-------
sphharm    Gauss-Legendre x trapezoid grid, real spherical harmonics, transforms (§3)
geometry   surface geometry, smooth quadrature weights, area, centroid, tau (§2.2, §3)
singular   weakly singular self-interaction operators by grid rotation (§3, §3.1)
farfield   off-body Stokeslet / traction / pressure sums (§2.1, §3.1)
nearfield  upsampled smooth rule for near body pairs (§3)
system     incident density, augmented second-kind system, solves, velocities (§2.2-§3.3)
timestep   quaternion RK4 evolution of centres and orientations (§3.3)
contact    contact forces between touching bodies (§3.3 contact force algorithm)
magnetic   magnetostatic potential, field and Maxwell traction of permeable bodies (§4)
fmm        fast multipole approximation of the off-body traction sum (the O(N) far field of §3.1)
mlp        FP64 reference of the warm-start network (forward, backward, Adam)

Every floating-point quantity is computed in float64.
"""
