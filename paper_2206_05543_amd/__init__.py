"""MI355X-native SPAI-smoothed geometric multigrid (arXiv 2206.05543)."""
