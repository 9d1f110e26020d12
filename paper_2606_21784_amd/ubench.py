"""Issue-rate microbenchmarks behind the engine's roofline (runs on the GPU).

    python -m paper_2606_21784_amd.ubench [out.json]

Each kernel runs 8 independent chains of one instruction per lane.  One workgroup per CU of
n = 1, 2, 4, 8 or 16 waves; per workgroup the kernel records shader-clock cycles and real-time
ticks of its loop (ended by a workgroup barrier, so the slowest wave counts).  Reported per
instruction and n: wave64 instructions per clock per CU (independent of the clock), lane
operations per CU per clock, and the shader clock the GPU ran at.
"""
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {"v_add_u32": 0, "v_xor_b32": 1, "v_bitop3_b32": 2, "v_mul_hi_u32": 3,
         "v_mul_lo_u32": 4, "v_mad_u64_u32": 5, "ds_add_u32_conflict_free": 6,
         "ds_add_u32_window66": 7, "v_fma_f32": 8, "v_fma_f64": 9}


def measure(iters=4096, reps=3):
    import torch
    lib = C.CDLL(os.path.join(HERE, "libcae_ubench.so"))
    lib.cae_ubench_run.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p,
                                   C.c_void_p, C.c_void_p]
    lib.cae_ubench_wallclock_khz.restype = C.c_int
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    wall_hz = lib.cae_ubench_wallclock_khz() * 1e3 or 100e6
    res = {"num_cu": ncu, "wallclock_hz": wall_hz, "iters": iters, "ops_per_iter": 8}
    for nw in (1, 2, 4, 8, 16):  # waves in the one workgroup per CU
        blocks = ncu
        threads = 64 * nw
        out = torch.empty(blocks * threads, dtype=torch.int32, device="cuda")
        clk = torch.zeros(2 * blocks, dtype=torch.int64, device="cuda")
        for name, k in KINDS.items():
            best = None
            for _ in range(reps):
                ms = C.c_float()
                it = iters // 4 if name.startswith("ds_") else iters
                rc = lib.cae_ubench_run(k, blocks, threads, it, out.data_ptr(), clk.data_ptr(),
                                        C.byref(ms))
                if rc != 0:
                    raise RuntimeError("ubench %s failed (%d)" % (name, rc))
                c = clk.cpu().numpy().reshape(-1, 2).astype(np.float64)
                cyc, ticks = float(np.median(c[:, 0])), float(np.median(c[:, 1]))
                row = {"ms": ms.value, "cycles": cyc, "ghz": cyc / (ticks / wall_hz) / 1e9,
                       "cu_ipc": it * 8.0 * nw / cyc,
                       "lane_ops_per_s": blocks * threads * it * 8.0 / (ms.value * 1e-3),
                       "kernel_cycles_at_ghz": ms.value * 1e-3 * cyc / (ticks / wall_hz)}
                row["lanes_per_cu_per_clk"] = 64.0 * row["cu_ipc"]
                if best is None or row["cycles"] < best["cycles"]:
                    best = row
            res["%s@%dw" % (name, nw)] = best
    return res


if __name__ == "__main__":
    r = measure()
    for k, v in r.items():
        if isinstance(v, dict):
            print("%-32s %6.3f wave-instr/clk/CU  %6.1f lanes/CU/clk  %.3f GHz  %.3g lane-op/s" %
                  (k, v["cu_ipc"], v["lanes_per_cu_per_clk"], v["ghz"], v["lane_ops_per_s"]))
    if len(sys.argv) > 1:
        with open(sys.argv[1], "w") as f:
            json.dump(r, f, indent=1)
