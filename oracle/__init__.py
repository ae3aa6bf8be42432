"""FP64 CPU oracle for the Voyager per-frame hot path (TEST INFRASTRUCTURE).

This package is test infrastructure, not product code. Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call it. It shares no code with the HIP library: it reads the same
seeded input arrays (from ``scenegen``) and nothing else.

It computes the PLAIN DEFINITIONS of what the method produces, in float64:

* ``lod``     - the LoD cut of Section 3.1 ("Cut Finding"): a node is on the
                cut when its projected size is below tau while its parent's is
                above; computed by brute force over every node. The paper's
                temporal-aware search (Section 4.1, Algorithm 1) claims a
                bit-accurate result, so it must reproduce this same set.
* ``sh``      - real spherical harmonics up to degree 3 (view-dependent colour).
* ``project`` - EWA culling & projection of each cut Gaussian (Section 3.1
                "Culling & Projection"), with the conventional 3DGS constants.
* ``render``  - per-pixel front-to-back alpha blending (Section 3.1
                "Rasterization"), alpha = min(0.99, theta * e^rho) (Eq. 3),
                Gaussians with alpha below alpha* skipped; no tiles, no
                preemptive filter (Section 4.2 claims the filter is lossless,
                so the filtered image must equal this one) and no LUT.
* ``grad``    - gradients of that image with respect to the Gaussians'
                parameters (blend decisions held fixed), by automatic
                differentiation of a torch float64 transcription on the CPU.

Every function marked "parity unpinned" in its docstring lacks an
independent pin; all others are pinned by tests/test_oracle_*.py.
"""
from . import lod, sh, project, render  # noqa: F401
# oracle.grad imports torch on use: `from oracle import grad`
