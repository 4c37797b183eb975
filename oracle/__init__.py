"""CPU oracle of the MPO bond update and the middle-MPO contraction.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may import it; the product path never does.  It shares no code with
the GPU path."""
