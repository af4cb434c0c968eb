"""Batched Bayesian identification of Schnakenberg reaction-diffusion
parameters on MI355X (gfx950): HIP kernels behind the C ABI of
include/rdbayes.h, with a thin Python binding (``api``).

Importing the package loads nothing; ``api`` loads librdbayes.so on first
use and raises if it is not built (there is no CPU fallback).
"""
