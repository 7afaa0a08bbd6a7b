"""Seeded synthetic inputs shared by tests, benchmark and smoke check."""
