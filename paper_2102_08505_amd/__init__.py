"""MI355X-native thresholded ELLPACK X^2 and SP2 purification (arXiv 2102.08505 hot path)."""
