"""Instruction rates behind the sweep's VALU roofline (include/pdg_rates.h):

    python -m paper_1611_06684_amd.rates [--iters N]

prints one JSON line: the measured rates of 32-bit adds (a full-rate
reference), v_mad_u64_u32 and whole Philox4x32-10 calls on the current GPU, and
what they imply in full-rate issue slots (against the nominal 256 CUs x 4 SIMDs
x 16 lanes x 2.4 GHz = 39.3 T lane-operations/s and against the measured add
rate).  The binding only marshals arguments; the loops run in libpdg.so.
"""
from __future__ import annotations

import argparse
import ctypes
import json

from . import pdg

EXPORTS = ["pdg_valu_rates"]
NOMINAL = 256 * 4 * 16 * 2.4e9


def pdg_valu_rates(device: int = 0, iters: int = 1 << 14):
    L = pdg.lib()
    f = L.pdg_valu_rates
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    out = (ctypes.c_double * 3)()
    rc = f(device, iters, out)
    if rc != 0:
        raise RuntimeError(f"pdg_valu_rates failed with status {rc}")
    return list(out)


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--iters", type=int, default=1 << 14)
    a = p.parse_args(argv)
    add, mad, philox = pdg_valu_rates(0, a.iters)
    print(json.dumps({
        "add_lane_ops_per_s": add, "mad64_lane_ops_per_s": mad, "philox_calls_per_s": philox,
        "nominal_lane_ops_per_s": NOMINAL,
        "add_frac_of_nominal": add / NOMINAL,
        "mad64_slots_per_op": add / mad,
        "philox_slots_per_call": add / philox,
        "philox_slots_per_call_nominal": NOMINAL / philox,
    }))


if __name__ == "__main__":
    main()
