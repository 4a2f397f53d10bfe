"""MI355X-native hot path of the block-based multiresolution Euler solver (arXiv 2012.04385)."""
