"""Measured ceilings of the GPU in use: FP64 FMA on the vector units, the FP64, FP32 and
int8 matrix cores, HBM read and copy bandwidth.  The thin-SVD rooflines quote these beside
the datasheet peaks (bench.py reads the JSON this writes).

Run on the GPU:  python -m paper_2603_11953_amd.peaks [--out profiles/peaks_mi355x.json]

Each probe (probe/peaks.hip, built into libgsvd_peaks.so) keeps independent dependency
chains in every lane of a grid that fills the device several times over; its rate is the
best of three timed launches of about 20-100 ms each, with HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_OUT = os.path.join(ROOT, "profiles", "peaks_mi355x.json")


def _lib():
    import torch  # noqa: F401 -- one HIP runtime for torch and the probe library
    path = os.path.join(HERE, "libgsvd_peaks.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build with paper_2603_11953_amd/build.py")
    L = ctypes.CDLL(path)
    L.probe_compute.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_void_p]
    L.probe_compute.restype = ctypes.c_int
    L.probe_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                             ctypes.c_void_p]
    L.probe_read.restype = ctypes.c_int
    return L


def _best_ms(torch, fn, reps=3):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def measure() -> dict:
    import torch
    L = _lib()
    dev = torch.device("cuda:0")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * 8
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    st = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    res = {}
    # (kind, iterations, work per wavefront per iteration, key, unit scale)
    probes = [(0, 200_000, 64 * 8, "fp64_valu_lane_tops"),    # FMAs (one lane-op each)
              (1, 20_000, 4 * 2048, "fp64_mfma_tflops"),      # 16x16x4 FP64: 2048 flops
              (2, 50_000, 4 * 2048, "fp32_mfma_tflops"),      # 16x16x4 FP32: 2048 flops
              (3, 200_000, 4 * 32768, "int8_mfma_tops")]      # 16x16x64 int8: 32768 ops
    for kind, iters, per_wave_iter, key in probes:
        def run():
            rc = L.probe_compute(kind, blocks, iters, out.data_ptr(), st)
            if rc != 0:
                raise RuntimeError(f"probe_compute({kind}) = {rc}")
        ms = _best_ms(torch, run)
        work = blocks * 4 * iters * per_wave_iter
        res[key] = round(work / (ms * 1e-3) / 1e12, 2)
    res["fp64_valu_tflops"] = round(2 * res["fp64_valu_lane_tops"], 2)
    n = (4 << 30) // 8  # 4 GiB
    buf = torch.ones(n, dtype=torch.float64, device=dev)
    rblocks = cus * 16
    rout = torch.empty(rblocks * 256, dtype=torch.float64, device=dev)

    def rd():
        rc = L.probe_read(buf.data_ptr(), n, rblocks, rout.data_ptr(), st)
        if rc != 0:
            raise RuntimeError(f"probe_read = {rc}")
    res["hbm_read_gbps"] = round(n * 8 / (_best_ms(torch, rd) * 1e-3) / 1e9, 1)
    half = n // 2
    src, dst = buf[:half], buf[half:]
    res["hbm_copy_gbps"] = round(2 * half * 8 / (_best_ms(torch, lambda: dst.copy_(src)) * 1e-3)
                                 / 1e9, 1)
    del buf
    return {"device": torch.cuda.get_device_name(0), "compute_units": cus, "peaks": res,
            "units": {"fp64_valu_lane_tops": "1e12 FP64 FMA lane-instructions/s",
                      "fp64_valu_tflops": "1e12 flop/s (FMA = 2)",
                      "fp64_mfma_tflops": "1e12 flop/s", "fp32_mfma_tflops": "1e12 flop/s",
                      "int8_mfma_tops": "1e12 int8 op/s", "hbm_read_gbps": "1e9 B/s read",
                      "hbm_copy_gbps": "1e9 B/s read + written (torch copy_)"},
            "datasheet": {"fp64_valu_tflops": 78.6, "fp64_mfma_tflops": 78.6,
                          "fp32_mfma_tflops": 157.3, "int8_mfma_tops": 5000.0,
                          "hbm_gbps": 8000.0},
            "command": "python -m paper_2603_11953_amd.peaks"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    r = measure()
    print(json.dumps(r))
    with open(args.out, "w") as f:
        json.dump(r, f, indent=1)


if __name__ == "__main__":
    main()
