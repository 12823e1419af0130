"""MI355X-native Klinkenberg lattice Boltzmann hot path (arXiv:1411.7051)."""
