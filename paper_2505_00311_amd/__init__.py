"""MI355X-native PDCS hot path (package root)."""
