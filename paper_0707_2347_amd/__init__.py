"""Exact Strassen-Winograd products over Z/pZ on MI355X (package placeholder)."""
