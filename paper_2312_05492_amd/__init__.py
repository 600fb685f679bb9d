"""MI355X-native G-Interp error-bounded compressor (cuSZ-i, arXiv 2312.05492)."""
