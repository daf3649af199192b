"""CPU oracle of the differentiable tile-based Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
It shares no code with the HIP path and never calls it.

The paper (On-the-fly Large-scale 3D Reconstruction from Multi-Camera Rigs)
renders its Gaussians with the differentiable rasterizer of 3D Gaussian
Splatting and updates Gaussian parameters by gradients (Sec. 3.3,
"Optimization"), with the colour carried by spherical harmonics; it does not
spell the image model out.  The oracle writes that image model down as a plain
definition:

* ``spec32``     FP32 visibility / depth / pixel-box decisions (the binning
                 rules), evaluated op by op in IEEE binary32, so that keys and
                 tile lists can be compared bit for bit.
* ``project64``  FP64 EWA projection of each Gaussian to a 2D mean, conic,
                 opacity and view-dependent colour.
* ``render64``   brute-force per-pixel front-to-back compositing in FP64, with
                 no tiles.
* ``grad64``     FP64 gradients by torch autograd through the same definition
                 with every discrete decision held fixed.
* ``binning``    the (view | tile | depth) keys and per-tile lists that the
                 definition implies.
* ``adam64``     the FP64 Adam recurrence used as the parameter step.
* ``loss64``     the L1 photometric loss and its gradient.
* ``fd``         central finite differences of the FP64 renderer.
"""
