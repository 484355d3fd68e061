"""MI355X-native micro-batch stream operators (LMStream, arXiv 2111.04289).

Submodules:

* ``lms``      -- ctypes binding of the C-ABI library ``liblms.so``
                  (include/lms.h): filter/project, windowed group-by,
                  stream-static hash join, MapDevice placement.
* ``datagen``  -- seeded synthetic micro-batches.
* ``build``    -- compiles the HIP sources for gfx950.

Importing the package loads nothing; ``paper_2111_04289_amd.lms`` loads the
library and raises if it is missing.
"""
