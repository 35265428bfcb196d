"""MI355X-native order-space MCMC for Bayesian-network structure learning.

The compute path lives in the HIP library ``libbnos.so`` built from ``csrc/``
(C-ABI declared in ``include/bnos.h``); ``bnos`` is its thin ctypes binding.
``datagen`` draws seeded synthetic inputs.  Importing this package does not
load the library; ``paper_1210_5128_amd.bnos`` does, and fails loudly when it
has not been built.
"""
