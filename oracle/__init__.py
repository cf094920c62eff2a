"""FP64 CPU oracle of the real-time transient hot path (Ruhe et al.,
"Detecting Dispersed Radio Transients in Real Time Using Convolutional
Neural Networks", arXiv:2103.15418).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke entry point and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library and
imports nothing from it.

It is a plain, slow, obviously correct numpy transcription of what the
method computes, evaluated in float64 on the float32 input values:

* ``qc``       quality control: band mean / RMS robust z-scores and the
               per-pixel running-statistics score (App. A);
* ``filters``  the Gaussian / box kernel and the masked, normalised
               centre/spread estimates C and S (Sec. 2.1.1);
* ``detect``   sigma thresholding with clip iterations and the 7x7
               maximum-filter peak map P = Q and Y (Sec. 2.1.1-2.1.2);
* ``catalog``  cross-band duplicate removal, association with the previous
               step, monitoring (Sec. 2.2);
* ``flux``     box-maximum flux per band, backward fill from cached images
               and the dynamic-spectrum window (Sec. 2.2, Fig. 3);
* ``cnn``      the parameter-inference network and its Cholesky head
               (Sec. 2.3.2-2.3.3);
* ``pipeline`` one stream's state across time steps, tying them together.

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (brute force, closed forms, invariants or an independent library
routine); see the module docstrings for the passage each follows.
"""

from .config import OracleConfig  # noqa: F401
from .pipeline import OracleStream  # noqa: F401
