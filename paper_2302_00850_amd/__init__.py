"""MI355X (gfx950) Wilson-Dirac hot path: HIP kernels behind a C ABI.

    from paper_2302_00850_amd import cola      # ctypes binding of libcola.so
    from paper_2302_00850_amd import synth     # seeded synthetic inputs

The binding is imported lazily so that input generation works without the
built library; every operator call goes through libcola.so.
"""
__all__ = ["cola", "synth", "build"]
