"""CPU oracle for the homomorphic linear-layer path of CryptoTrain (arXiv 2409.16675).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package; the product library never
does, and this package never imports the product.

Contents:
  * ``core``    -- ctypes wrappers over ``oracle.c`` (exact modular arithmetic,
                   schoolbook ring product, transform definition, term-list MAC);
  * ``pyref``   -- a pure-Python big-integer reference for tiny rings, used to pin
                   the C code;
  * ``packing`` -- the correlation-aware packings of Section 3.3 (Eq. 1, Eq. 2)
                   and the readings used for channels, weight gradients and FC;
  * ``bfv``     -- test-only BFV-style encryption / decryption with CRT;
  * ``plain``   -- plaintext integer convolution, weight gradient and mat-vec.
"""
