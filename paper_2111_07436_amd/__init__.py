"""MI355X-native batched stiff multiphase chemistry solver (CAMP hot path).

Submodules are imported lazily: ``workloads`` (seeded synthetic inputs) needs no GPU
library; ``camp`` (the ctypes binding to the HIP library) loads ``libcamp.so`` and fails
loudly when it is missing.
"""
