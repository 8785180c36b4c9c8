"""MI355X value iteration for perishable-inventory MDPs.

`paper_2303_10672_amd.pvi` is the ctypes binding of libpvi.so (include/pvi.h);
`paper_2303_10672_amd.build` compiles the library with hipcc for gfx950.
"""
