"""Plain FP64 CPU reference ("oracle") for the BlockMGARD hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product library (``paper_2609_00205_amd``) never imports, links or calls it,
and this package imports nothing from the product library: the two share no
code, tables or constants.

Modules
-------
``mgard``    nested grids, 1D operators, global and In-cache Block levels, the
             hybrid hierarchy, padding, and the adjoint (transpose) maps.
``roi``      block tolerance maps, conservative propagation (Eq. 2), the
             per-level error budget and the reciprocal quantizer.
``paper8``   the paper's own block form: disjoint 8^3 blocks whose 5^3
             coarse outputs are re-assembled into the next level's blocks.
``huffman``  canonical Huffman code lengths, chunked MSB-first bitstream.
``selector`` the throughput model (Eq. 1) and the (L, M) selector of
             Algorithm 1.

Everything is written from the paper's text (sections II-B, IV-A..IV-D,
V-A) and the readings stated in each module's header where the paper is
silent; every function cites the passage it follows.
"""
