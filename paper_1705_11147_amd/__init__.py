"""MI355X-native k-mer analysis (HipMer / Meraculous, arXiv 1705.11147).

Submodules:
  abi    -- ctypes binding of the C ABI in include/hm_kmer.h (libhm_kmer.so)
  kmer   -- device buffers + the ordered C-ABI calls of the path
  synth  -- seeded synthetic genomes and reads (no k-mer arithmetic)

Importing the package loads nothing; the HIP library is loaded on first use
and its absence is an error (there is no CPU fallback).
"""

__all__ = ["abi", "kmer", "synth"]
