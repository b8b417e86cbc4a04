"""Plain CPU oracle of the fusion hot path (test infrastructure only)."""
