"""MI355X-native state-vector quantum circuit simulator (qHiPSTER's problem,
arXiv:1601.07195, on one gfx950 GPU).

    paper_1601_07195_amd.qs      ctypes binding of libqs.so (the C ABI in
                                 include/qs.h); raises ImportError when the
                                 library has not been built
    paper_1601_07195_amd.build   builds libqs.so with hipcc for gfx950
"""
