"""lpbatch for MI355X: batched dense-tableau simplex (Gurung & Ray, arXiv:1802.08557).

``paper_1802_08557_amd.lpbatch``   -- ctypes binding of the C-ABI library
``paper_1802_08557_amd.workloads`` -- seeded synthetic LP batches

Importing the package loads nothing; the HIP library is opened on first use of
``lpbatch``.
"""
