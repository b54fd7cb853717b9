"""MI355X-native two-component colour-gradient D3Q19 lattice Boltzmann (arXiv 2005.12764 hot path)."""
