"""Seeded synthetic inputs for the calibrated FFT-correlator.

This package only draws random numbers and builds the instrument model's
inputs (sky, gains, noise, voltages; and, in `visibilities`, the
visibility-level simulation of the paper's Sec. 3).  It contains none of the correlator's
or the calibrator's arithmetic, so both the CPU oracle and the HIP path can
consume the very same bytes without sharing any of the method's code.
"""
from .generate import (WORKLOADS, Workload, sky_power, unit_gains, unit_voltages,
                       quantise_ci4, pack_ci4, unpack_ci4, workload_voltages)

__all__ = ["WORKLOADS", "Workload", "sky_power", "unit_gains", "unit_voltages",
           "quantise_ci4", "pack_ci4", "unpack_ci4", "workload_voltages"]
