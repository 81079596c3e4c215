"""MI355X-native FR residual for ACM with hyperbolised diffusion (arXiv:2107.14027)."""
