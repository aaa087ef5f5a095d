"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This package holds no arithmetic of the sampling method: it writes weight
files (random initialisation of a declared architecture), synthetic
fBm-shaped terrain latents and query streams.  Both the HIP path and the
oracle consume what it writes; neither is imported here.
"""
