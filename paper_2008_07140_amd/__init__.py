"""Full-amplitude quantum state-vector simulator for AMD MI355X (gfx950).

The compute path is the C-ABI library ``libqs.so`` (hand-written HIP
kernels); ``paper_2008_07140_amd.qs`` is its thin ctypes binding and
``paper_2008_07140_amd.circuits`` the seeded synthetic circuit generator.
"""
