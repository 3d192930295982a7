"""Accumulation-error bounds shared by the MFMA probe test and the layer-wise
low-precision tests, as fractions of the sum of absolute products.

FP32 and BF16 MFMAs accumulate in FP32: at most (K + 1) unit roundoffs of
2^-24 for K products per output (BF16 products are exact in FP32, FP32
products round once). The 16x16x128 FP8 (f8f6f4) MFMA adds its 128 products
with less precision than FP32. On MI355X, over random full-range e4m3fn
operands (products spanning about 2^35), one instruction's error reached
1.96e-4 of the sum of |products| with mixed signs and 2.97e-4 with one sign
(5.5e-4 and 1.0e-3 of the largest |product|); chains of ten stayed below
1.1e-4. tests/test_gpu_mfma.py measures these and asserts FP8_ACC_REL, twice
the largest, on every tile it runs.
"""
U32 = 2.0 ** -24
FP32_ACC_REL = 17 * U32   # 16 products per FP32 chunk (four 16x16x4 MFMAs)
BF16_ACC_REL = 33 * U32   # 32 products per 16x16x32 MFMA
FP8_ACC_REL = 6e-4        # per 16x16x128 f8f6f4 MFMA or chain of them (measured max 2.97e-4)
