"""MI355X-native Rayleigh-Sommerfeld integral (RSI) quasi-Monte-Carlo beam model.

The compute path is the HIP library ``librsi.so`` (C ABI in ``include/rsi.h``);
``rsi`` is its thin Python binding.  Importing this package loads nothing; the
library is loaded on first use and its absence is an error (there is no fallback).
"""
__all__ = ["rsi", "workloads"]
