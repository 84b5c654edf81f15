"""MI355X-native eddy-current A-V solver (HIP kernels behind a C ABI).

`paper_1602_03207_amd.eddy` holds the ctypes binding of libeddy.so;
`paper_1602_03207_amd.build` compiles it for gfx950.
"""
