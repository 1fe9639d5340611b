"""MI355X-native HODLR factorization and solve (hand-written HIP for gfx950).

The compute path lives in the C-ABI library ``libhodlr.so`` (sources in
``csrc/``, interface in ``include/hodlr.h``); this package only marshals
arguments to it.  Import ``paper_2208_06290_amd.hodlr`` for the Python API.
"""
