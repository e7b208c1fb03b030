"""k-clique-core densest-subgraph discovery on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libdsd.so`` (C ABI in include/dsd.h);
``paper_1906_00341_amd.dsd`` is its thin Python binding and
``paper_1906_00341_amd.synth`` draws the seeded synthetic input graphs.
"""
