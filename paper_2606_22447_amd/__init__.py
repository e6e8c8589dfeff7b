"""MI355X-native batched Atari VCS emulation (hard and soft straight-through forms).

The hot path runs in hand-written HIP kernels behind the C-ABI declared in
``include/vcs.h``; this package holds the seeded workload generator
(:mod:`.inputs`), the thin ctypes binding (:mod:`.binding`) and the torch-facing
wrappers (:mod:`.vcs`).
"""
