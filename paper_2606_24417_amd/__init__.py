"""MI355X (gfx950) Super Bloom filter for DNA k-mers: the sequence-native
insert and query path (2-bit encoding, rolling minimizer and s-mer hashing,
super-k-mer sharding, atomic-OR insert, leader-load query) behind the C ABI
of include/sbf.h, with a thin ctypes binding."""

from .sbf import (SBF_E_BUSY, SBF_E_DEVICE, SBF_E_INVAL, SBF_E_NOMEM, SBF_OK, VARIANT_AUTO, VARIANT_GENERIC,
                  VARIANT_PARAM, VARIANT_ROLLING, VARIANT_WIDE, Filter, Graph, SBFError, Server, autotune_geometry,
                  last_error, lib)

__all__ = ["Filter", "Graph", "Server", "SBFError", "lib", "last_error", "SBF_OK", "SBF_E_INVAL", "SBF_E_NOMEM", "SBF_E_DEVICE", "SBF_E_BUSY",
           "VARIANT_AUTO", "VARIANT_ROLLING", "VARIANT_GENERIC", "VARIANT_WIDE", "VARIANT_PARAM",
           "autotune_geometry"]
