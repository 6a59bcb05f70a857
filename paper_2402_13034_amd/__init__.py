"""MI355X-native RIS-aware ray tracer (arXiv 2402.13034 hot path)."""
