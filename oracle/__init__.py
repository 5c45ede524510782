"""CPU oracle of the SA-AMG setup and solve (test infrastructure only)."""
