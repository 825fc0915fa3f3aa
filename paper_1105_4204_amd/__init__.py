"""Constant-time trigonometric bilateral filter on MI355X (gfx950).

Placeholder while the native library is built; the binding is added below.
"""
