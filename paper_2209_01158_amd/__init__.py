"""MI355X-native decoupled multicontinuum flow solver (HIP kernels behind a C ABI).

The binding lives in ``paper_2209_01158_amd.mcdec`` (imported on demand, so that building
or inspecting the package does not need the compiled library).
"""
__version__ = "0.1.0"
