"""Seeded synthetic inputs for the PRENOM per-object NeRF training step.

This package generates inputs only: architectures, analytic scenes with their
closed-form ground truth, pinhole cameras and rays, prior density grids,
initial parameters and the random numbers the sampler consumes.  It holds none
of the method's arithmetic (no sampling, encoding, MLP, compositing, loss or
optimiser code); both the CPU oracle tests and the GPU path consume its
outputs.
"""
