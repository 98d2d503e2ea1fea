"""Timing-aware 4-value gate-level re-simulation on AMD MI355X (gfx950)."""
