"""Accumulation-error bounds shared by the MFMA probe test and the layer-wise
low-precision tests, as fractions of the sum of absolute products.

FP32 and BF16 MFMAs accumulate in FP32: at most (K + 1) unit roundoffs of
2^-24 for K products per output (BF16 products are exact in FP32, FP32
products round once). The 16x16x128 FP8 (f8f6f4) MFMA adds its 128 products
with less precision than FP32: on random full-range e4m3fn operands (products
spanning about 2^35) one instruction's error reached 1.96e-4 of the sum of
|products| (about 2^-12.3) on MI355X; tests/test_gpu_mfma.py measures it and
asserts FP8_ACC_REL, twice that, on every tile it runs, for single
instructions and for chains of ten (a conv's K steps).
"""
U32 = 2.0 ** -24
FP32_ACC_REL = 17 * U32   # 16 products per FP32 chunk (four 16x16x4 MFMAs)
BF16_ACC_REL = 33 * U32   # 32 products per 16x16x32 MFMA
FP8_ACC_REL = 4e-4        # per 16x16x128 f8f6f4 MFMA or chain of them (measured max 1.96e-4)
