"""FP64 CPU oracle -- test infrastructure only (tests, smoke check and the
benchmark's CPU-baseline leg).  The library never imports it."""
