"""Serial CPU oracle for the Morse-Smale hot path -- TEST INFRASTRUCTURE ONLY.

Used by tests/, the smoke check and the benchmark's CPU-baseline leg; never by
the product path."""
