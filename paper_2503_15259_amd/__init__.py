"""MI355X-native PSCA device activity detection (arXiv 2503.15259)."""
