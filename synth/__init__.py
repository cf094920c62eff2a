"""Seeded synthetic input streams shared by the oracle's tests, the device
tests and the benchmark.  Holds no arithmetic of the detection method."""

from .sky import (C_DM, FWHM_PX, SIGMA_PSF, Source, Stream, StreamSpec,  # noqa: F401
                  arrival_times, boxcar_overlap, sky_mask, spec_instrument,
                  spec_serving_streams, spec_streaming, spec_tiny, two_group_freqs)
from .weights import cnn_weights  # noqa: F401
