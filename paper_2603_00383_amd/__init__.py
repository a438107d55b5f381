"""MI355X-native stress-transfer path of the divide-and-conquer elastodynamic SEAS
method: HIP library (csrc/, built to libseas.so) and its ctypes binding."""
from ._seas import (FIELDS, SEAS_BF16, SEAS_F16, SEAS_F32, SEAS_F64, Operator, SeasError, Server, State, lib)  # noqa: F401
