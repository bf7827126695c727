"""MI355X-native bilayer minimum-mode kernel (arXiv 2509.26269)."""
