"""CPU oracle of the SDC-resilient compressor: test infrastructure only."""
