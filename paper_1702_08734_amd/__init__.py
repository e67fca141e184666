"""MI355X-native exact k-NN and IVFADC search (HIP kernels behind a C ABI).

Importing the package loads nothing; the compiled library is opened on the
first call into :mod:`paper_1702_08734_amd.api`, which raises if it is
missing.
"""
