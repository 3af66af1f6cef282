"""FP64 CPU oracle of the D2IP fitting iteration (arXiv 2507.14046).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark import this package; the GPU
library never calls it and shares no code with it.  Everything here is plain
NumPy in float64, written from the paper's definitions:

* ``net``  - the image prior phi(theta | Z) (Eq. (3), Sec. III-D) and its exact
             reverse-mode gradient;
* ``fit``  - the data term of Eq. (4), Adam, the TPP frame schedule
             (Eqs. (5), (9)) and the read-out;
* ``tv``   - the 4D-TV regulariser of Eqs. (11)-(14);
* ``dwsep``- the depthwise-separable 3D convolution of the lightweight
             backbone (Sec. III-D) and its gradients;
* ``se``   - the Squeeze-and-Excitation unit of the 3D-FastResUNet
             (Sec. III-D) and its gradients.

Parity pins (tests/test_oracle_*.py): central finite differences, brute-force
7-loop convolution, torch CPU float64 library operations, adjoint identities,
LayerNorm invariants, Adam closed forms, the least-squares limit of gradient
descent on the data term.  Nothing pins the whole multi-iteration trajectory
against the paper itself (the paper prints no worked example): "parity
unpinned" for the composed trajectory beyond those piecewise pins.
"""
from . import net, fit

__all__ = ["net", "fit"]
