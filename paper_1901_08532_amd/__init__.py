"""Hermite-6 direct N-body on one MI355X: package root."""
