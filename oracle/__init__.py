"""FP64 CPU oracle for HO-DMAS beamforming (test infrastructure only)."""
