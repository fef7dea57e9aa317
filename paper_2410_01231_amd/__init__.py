"""MI355X-native proximity-graph build path (arXiv 2410.01231).

The compute path is the C-ABI library ``libpg.so`` (hand-written HIP kernels
for gfx950); ``paper_2410_01231_amd.pg`` is its thin Python binding.  Nothing
is imported here, so the seeded input generators in ``datagen`` can be used
without the library: ``from paper_2410_01231_amd import pg`` loads it.
"""
