"""FP64 CPU oracle of the ECsim particle hot path (test infrastructure only)."""
