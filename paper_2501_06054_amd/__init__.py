"""MI355X (gfx950) small-angle neutron scattering sample tracer.

- ``paper_2501_06054_amd.sans``: ctypes binding of libsans (include/sans.h);
- ``paper_2501_06054_amd.workloads``: seeded synthetic inputs;
- ``paper_2501_06054_amd.build``: builds libsans.so in-tree with hipcc.
"""
