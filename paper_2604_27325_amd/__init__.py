"""Batched small symmetric eigendecomposition on MI355X (binding placeholder)."""
