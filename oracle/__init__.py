"""Plain FP64 CPU oracle of the sliding-mesh mortar operator: test infrastructure only."""
