"""CRSH (Coherent Ray-Space Hierarchy) secondary-ray path on MI355X.

``crsh``      ctypes binding of the C-ABI in include/crsh.h (libcrsh.so)
``pipeline``  the five stages chained on one stream with torch-owned memory
``build``     compiles libcrsh.so for gfx950
"""
