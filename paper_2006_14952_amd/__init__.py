"""MI355X-native truncated-FMM short-range gravity (placeholder, binding added below)."""
