"""MI355X-native per-patch ideal-MHD update (MHDTVD fluxes, CTU predictor and
constrained transport over batches of ghosted patches), after Mendygral et al.
2017 (WOMBAT), Sect. 5.2 and Appendix A.

    paper_1701_07452_amd.wmb     ctypes binding of libwmb.so (the HIP library)
    paper_1701_07452_amd.inputs  seeded synthetic inputs and patch tilings
    paper_1701_07452_amd.build   hipcc build of libwmb.so for gfx950
"""
