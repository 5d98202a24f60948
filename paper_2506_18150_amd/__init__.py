"""MI355X (gfx950) library for the CKKS plaintext-matrix x ciphertext product
behind HE-LRM's encrypted embedding lookups (arXiv 2506.18150).

The compute path is libhelrm.so (HIP kernels behind the C ABI in
include/helrm.h); ``binding`` marshals arguments to it, ``params``,
``encoding``, ``planner`` and ``client`` prepare its inputs, ``session``
ties them together, ``serving`` runs the request loop.
"""
