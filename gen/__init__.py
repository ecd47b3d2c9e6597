"""Seeded input generators (no hafnian arithmetic)."""
