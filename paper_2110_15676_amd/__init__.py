"""MI355X-native algebraic flux correction (AFC) for P1/Q1 CDR discretizations.

The compute path is the HIP library libafc.so (C ABI in include/afc.h); the
Python module `afc` is a thin ctypes binding with the same entry-point names.
`inputs` builds seeded synthetic problem instances.  Importing this package
loads nothing; `paper_2110_15676_amd.afc` loads the library on first use and
raises if it is missing.
"""
