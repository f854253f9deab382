"""MI355X (gfx950) implementation of the greedy rank-one ALS + Galerkin
solver for spatial connectome regression (Kuerschner, Dolgov, Harris &
Benner).  The solver lives in the HIP library libconnreg.so (C ABI in
include/connreg.h); ``connreg`` is its ctypes binding and ``synth`` draws
the seeded synthetic inputs."""

__all__ = ["connreg", "synth"]
