"""hisalog: semi-naive Datalog on one AMD MI355X over hash-indexed sorted
arrays.  The compute lives in libhisalog.so (hand-written gfx950 HIP
kernels behind the C ABI of include/hisalog.h); this package is its
Python binding."""

from .hisalog import (EXPORTS, LIB_PATH, Engine, HlError, RunStats, evaluate,  # noqa: F401
                      lib)
