"""MI355X-native space-charge field path of OuroborosBEM (arXiv 2110.09214).

The compute path is the HIP library libobem.so (C ABI declared in
include/obem.h); this package holds its thin ctypes binding (`binding`), the
torch.autograd wrapper of the field evaluation (`autograd`) and the seeded
synthetic workloads (`workloads`).  Importing the package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
