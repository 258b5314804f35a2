"""Adjoint of the implicit step (oracle) -- filled in below."""
