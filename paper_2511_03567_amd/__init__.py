"""MI355X-native spin-free RIC-MRCCSD residual engine (HIP kernels behind a C ABI)."""
