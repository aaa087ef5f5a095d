"""Plain FP64 CPU oracle for lazy InfiniteDiffusion sampling.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP path (its own weight-file reader, noise hash, window indexing, UNet,
sampler and Laplacian decode) so that agreement between the two means
something.

The oracle computes the *definition* of the method rather than the lazy,
cached algorithm: the seed fixes J_T (seeds paragraph, formal appendix), every
later J_t is the InfiniteDiffusion update (Eq. 2 / its formal restatement)
applied on a finite canvas that covers the query's dependency cone, and the
Laplacian decode follows Sec. 5.2 with the signed square-root inverse of the
signed-sqrt appendix.  Everything is float64 except the noise hash, whose
float32 operations are part of its specification (oracle.noise).

Parity status per function is listed in each module's header; a function with
no independent pin says "parity unpinned" there.
"""
