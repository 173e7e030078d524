"""MI355X-native free surface lattice Boltzmann (FSLBM) hot path."""
