"""MI355X (gfx950) implementation of the USP-FPM particle step for diatomic
gas (Kim & Jun, arXiv 2508.05642): hand-written HIP kernels behind the C ABI
of include/usp.h, with a thin ctypes binding in :mod:`.usp`."""
