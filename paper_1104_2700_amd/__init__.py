"""MI355X-native fourth-order Hermite force/jerk sweep with block timesteps.

The compute path is the HIP library ``libhermite.so`` (built from
``csrc/``) behind the C ABI declared in ``include/hermite.h``.  This package
only marshals arguments to it (``hermite``), generates seeded synthetic
inputs (``inputs``) and builds the library (``build``).  Importing the
package does not load the library; ``paper_1104_2700_amd.hermite`` does,
and fails loudly if it is missing.
"""
__all__ = ["inputs", "hermite", "build"]
