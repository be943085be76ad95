"""MI355X-native multi-case element-by-element (EBE) finite-element solver.

The compute path is a C-ABI HIP library (``include/ebe.h``) built for gfx950;
``paper_1710_08679_amd.ebe`` is its thin Python binding (argument
marshalling only).  ``meshgen`` builds seeded synthetic inputs.
"""
__all__ = ["ebe", "meshgen"]
