"""FP64 CPU oracle (test infrastructure only; see vdamp_ref's header)."""
