"""MI355X-native P-DFS / greedy weighted-set-cover (arXiv 2603.16721).

The compute path lives in the HIP library ``libpdfs.so`` built from
``csrc/``; ``pdfs`` is its ctypes binding.  ``synth`` generates seeded
synthetic cohorts.  Importing the package does not load the library.
"""
