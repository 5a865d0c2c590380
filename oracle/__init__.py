"""FP64 CPU oracle of the SDF photon random walk -- test infrastructure only."""
