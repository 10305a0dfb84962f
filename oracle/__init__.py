"""CPU oracle for the 3DGS render + NCC relocalisation hot path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct
NumPy statement of what the GPU library computes. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code, header, constant table or helper with the HIP
library in ``paper_2403_11367_amd``, and it never imports that package.

What each module follows (paper: "3DGS-ReLoc", arXiv 2403.11367):

* ``gaussians``  Sec. III-A, Gaussian parameters: Sigma = R S S^T R^T with
                 R = q2R(q) (quaternion w first) and S = diag(s).
* ``project``    Sec. III-A, Eq. 3 and Eq. 4: world-to-camera transform W_t,
                 pinhole projection m(mu) and its Jacobian J, screen-space
                 covariance J W Sigma W^T J^T (top-left 2x2), its inverse,
                 the 3-sigma pixel rectangle and the tile rectangle.
* ``keys``       Sec. III-A ("sorted by depth"): per-tile depth keys and the
                 reference order (tile, depth bits, Gaussian index).
* ``blend``      Eq. 1, Eq. 2 and Eq. 5: front-to-back compositing of colour
                 and depth with footprint q_i = o_i * exp(-d^2 / 2).
                 A tiled form and a brute-force per-pixel form.
* ``ncc``        Eq. 10: zero-mean normalised cross-correlation.
* ``crop``       Sec. III-B2: 2D voxel grid keyed by cell id and a radius
                 query around the prior camera centre (brute force over
                 cells, which is the plain definition of the KD-tree query).
* ``search``     Sec. III-C1: brute-force search = argmax of NCC over the
                 candidate renders (ties to the lowest index).

Readings of points the paper leaves open (all binding on both sides):

* Eq. 2's normalisation factor 1/(|J^-1||W^-1|) is read as 1 and the
  Gaussian as unnormalised, so q in [0, 1] as Eq. 1's transmittance needs.
* mu-hat in Eq. 2 is the projected pixel mean (first two entries of m(mu)).
* W in Eq. 3 is the rotation part of W_t; J is the 2x3 pixel-unit Jacobian
  at t = W mu with the normalised coordinates clamped to 1.3x the half field
  of view (clamp used in J only).
* Screen covariance dilation eps = 0.3 px^2 on both diagonal entries.
* A pair contributes only where d^2 <= 9, alpha = min(0.99, q) and
  alpha >= float32(1/255); compositing stops after the layer that takes the
  transmittance below 1e-4 (that layer counts).
* Near plane: cull unless t_z > 0.2. Background 0 for colour and depth.
  Depth is the camera-space z of the mean, not divided by coverage (Eq. 5).
* Pixel (i, j) is sampled at (i + 0.5, j + 0.5); tile id = ty * tiles_x + tx.
* Grey for NCC = 0.299 R + 0.587 G + 0.114 B; NCC = 0 if either image has
  zero variance.

The geometry and key steps run in IEEE float32 with a fixed operation order
(NumPy float32 never fuses multiply-adds), so the GPU can match the records
and keys bit for bit. Compositing and NCC run in float64.
"""
from . import gaussians, project, keys, blend, ncc, crop, search  # noqa: F401
