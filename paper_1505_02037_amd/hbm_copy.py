"""Plain device-to-device copy of a known size (include/hbm_probe.h).

Two uses: the achievable-bandwidth ceiling of the card (a copy moves each byte
once in and once out), and the calibration kernel for the HBM traffic counters
(FETCH_SIZE / WRITE_SIZE of a copy of B bytes each way should read B).

    python paper_1505_02037_amd/hbm_copy.py [--gib 4] [--reps 20]
    python paper_1505_02037_amd/hbm_copy.py --reread   (first vs second read, 16 MiB .. 4 GiB)
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhbmprobe.so")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=4.0)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-only", action="store_true", help="only the copy (counter calibration runs)")
    ap.add_argument("--reread", action="store_true", help="re-read vs cold read over a range of sizes")
    args = ap.parse_args()
    lib = ctypes.CDLL(LIB)
    for f in (lib.hbm_copy_probe, lib.hbm_read_probe):
        f.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.hbm_reread_probe.argtypes = [ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    if args.reread:
        for mib in (16, 32, 64, 128, 192, 256, 384, 512, 1024, 4096):
            nb = mib << 20
            hot, cold = ctypes.c_double(), ctypes.c_double()
            rc = lib.hbm_reread_probe(nb, 4 << 30, 5, ctypes.byref(hot), ctypes.byref(cold))
            if rc != 0:
                print(json.dumps({"error": rc, "MiB": mib}))
                return 1
            print(json.dumps({"MiB": mib, "GBps_reread": nb / (hot.value * 1e-3) / 1e9,
                              "GBps_cold": nb / (cold.value * 1e-3) / 1e9}), flush=True)
        return 0
    nbytes = int(args.gib * (1 << 30)) // 64 * 64
    ms, msr = ctypes.c_double(), ctypes.c_double()
    rc = lib.hbm_copy_probe(nbytes, args.reps, ctypes.byref(ms))
    if rc == 0 and not args.copy_only:
        rc = lib.hbm_read_probe(nbytes, args.reps, ctypes.byref(msr))
    if rc != 0:
        print(json.dumps({"error": rc}))
        return 1
    out = {"copy_bytes_each_way": nbytes, "ms_per_copy": ms.value,
           "GBps_read_plus_write": 2 * nbytes / (ms.value * 1e-3) / 1e9}
    if not args.copy_only:
        out.update({"ms_per_read": msr.value, "GBps_read_only": nbytes / (msr.value * 1e-3) / 1e9})
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
