"""MI355X implementation of the per-generation update of sPEGG's
individual-based eco-evolutionary model (Okamoto & Amarasekare).

``spegg`` is the binding of the HIP library (``libspegg.so``);
``workloads`` holds the seeded synthetic workloads.  Importing the package
loads nothing; ``spegg.load()`` does, and fails if the library is missing.
"""
