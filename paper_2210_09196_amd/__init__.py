"""MI355X-native 5G PUSCH lower-PHY receive chain.

OFDM-demodulation FFTs, beamforming, least-squares channel estimation and the
per-subcarrier MMSE MIMO solve (Gram + sigma^2 I, Cholesky, forward/back
substitution), as hand-written gfx950 HIP kernels behind the C ABI declared in
include/pusch.h.  The Python binding lives in `paper_2210_09196_amd.pusch`.
"""
