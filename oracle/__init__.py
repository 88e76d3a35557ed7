"""FP64 CPU oracle of the B-TriRT D2Q9 scheme: test infrastructure only."""
