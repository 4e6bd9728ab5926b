"""MI355X-native neural receiver (CGNN) for the 5G NR PUSCH: HIP kernels behind the libnrx C ABI."""
