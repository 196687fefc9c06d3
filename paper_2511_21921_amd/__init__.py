"""MI355X CRKSPH neighbour-pair passes (HIP library libcrk.so + ctypes binding)."""
from .crk import (CUBIC_SPLINE, FP32, FP64, WENDLAND_C4, Context, CrkError,  # noqa: F401
                  CRKSPHFunction, Params, lib)
