"""Issue-rate microbenchmarks behind the engine's roofline (runs on the GPU).

    python -m paper_2606_21784_amd.ubench [out.json]

The single-instruction kernels run 8 independent chains of one instruction per lane.  Three
more time the engine's generator in the form the engine issues it: v_mad_u64_u32 with a scalar
multiplier (mad_u64_const), Philox4x32-10 rounds on two counters per lane (philox_rounds: 2
products and 2 three-input xors per round and counter), and the engine's own per-agent NOISE
order code from cae_philox.h (gen_noise_events: two rows of 64 agents per wave and pass, the
order folded into a register instead of the LDS atomic).  One workgroup per CU of n = 1, 2, 4,
8 or 16 waves; per workgroup the kernel records shader-clock cycles and real-time ticks of its
loop (ended by a workgroup barrier, so the slowest wave counts).  Reported per kernel and n:
wave64 operations per clock per CU (instructions, or agent events for gen_noise_events;
independent of the clock), lane operations per CU per clock, and the shader clock the GPU ran at.
``summary`` derives the issue costs the roofline uses.
"""
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {"v_add_u32": 0, "v_xor_b32": 1, "v_bitop3_b32": 2, "v_mul_hi_u32": 3,
         "v_mul_lo_u32": 4, "v_mad_u64_u32": 5, "ds_add_u32_conflict_free": 6,
         "ds_add_u32_window66": 7, "v_fma_f32": 8, "v_fma_f64": 9,
         "mad_u64_const": 10, "philox_rounds": 11, "gen_noise_events": 12, "ds_rw_b64_words": 13,
         "gen_noise_events_4rows": 14, "v_add_u32_with_s_mul_i32": 15, "s_mul_i32": 16}
# operations per lane and loop iteration of each kernel
OPS_PER_ITER = {k: 8 for k in KINDS}
OPS_PER_ITER.update({"philox_rounds": 80, "gen_noise_events": 2, "ds_rw_b64_words": 16,
                     "gen_noise_events_4rows": 2})


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
                if name in ("philox_rounds", "gen_noise_events", "gen_noise_events_4rows"):  # ~80 per iteration
                    it = max(8, iters // 8)
                rc = lib.cae_ubench_run(k, blocks, threads, it, out.data_ptr(), clk.data_ptr(),
                                        C.byref(ms))
                if rc != 0:
                    raise RuntimeError("ubench %s failed (%d)" % (name, rc))
                c = clk.cpu().numpy().reshape(-1, 2).astype(np.float64)
                cyc, ticks = float(np.median(c[:, 0])), float(np.median(c[:, 1]))
                ops = OPS_PER_ITER[name]
                row = {"ms": ms.value, "cycles": cyc, "ghz": cyc / (ticks / wall_hz) / 1e9,
                       "cu_ipc": it * float(ops) * nw / cyc,
                       "lane_ops_per_s": blocks * threads * it * float(ops) / (ms.value * 1e-3),
                       "kernel_cycles_at_ghz": ms.value * 1e-3 * cyc / (ticks / wall_hz)}
                row["lanes_per_cu_per_clk"] = 64.0 * row["cu_ipc"]
                if best is None or row["cycles"] < best["cycles"]:
                    best = row
            res["%s@%dw" % (name, nw)] = best
    res["summary"] = summary(res)
    return res


def summary(res, nw=16):
    """Issue costs in full-rate slots (one slot = one lane of a full-rate 32-bit VALU instruction;
    v_add_u32 sets the full rate) at n = nw waves per CU:
      mad_const_slots:     v_mad_u64_u32 in the engine's form, alone;
      mad_in_mix_slots:    the same product inside Philox rounds, taking the three-input xor at its
                           own measured cost;
      gen_slots_per_event: slots one agent event of the engine's NOISE order code occupies
                           (generator, range reductions, clamp, book word);
      gen_events_per_clk_cu: its agent events per clock per CU;
      lds_window_lane_atomics_per_clk_cu: ds_add_u32 lane-operations per clock per CU in a
                           66-word window (the engine's aggregation pattern);
      lds_rw_b64_lane_words_per_clk_cu: 32-bit words per clock per CU moved by the clearing's
                           access form (ds_read_b64 and ds_write_b64 of (bid, ask) pairs)."""
    g = lambda k: res["%s@%dw" % (k, nw)]["cu_ipc"]
    full = g("v_add_u32")
    xor3 = full / g("v_bitop3_b32")
    round_slots = full / (g("philox_rounds") / 80.0) / 80.0 * 4.0  # slots per round and counter
    out = {"full_rate_wave_instr_per_clk_cu": full,
           "bitop3_slots": xor3,
           "mul_hi_slots": full / g("v_mul_hi_u32"),
           "mad_vvv_slots": full / g("v_mad_u64_u32"),
           "mad_const_slots": full / g("mad_u64_const"),
           "mad_in_mix_slots": (round_slots - 2.0 * xor3) / 2.0,
           "gen_events_per_clk_cu": 64.0 * g("gen_noise_events"),
           "gen_slots_per_event": 64.0 * full / (64.0 * g("gen_noise_events")),
           "gen4_events_per_clk_cu": 64.0 * g("gen_noise_events_4rows"),
           "lds_window_lane_atomics_per_clk_cu": 64.0 * g("ds_add_u32_window66"),
           "lds_conflict_free_lane_atomics_per_clk_cu": 64.0 * g("ds_add_u32_conflict_free"),
           "lds_rw_b64_lane_words_per_clk_cu": 64.0 * g("ds_rw_b64_words"),
           "ghz": res["v_add_u32@%dw" % nw]["ghz"]}
    # one wave per SIMD (4 waves per CU): what a single wave can issue per SIMD clock, VALU alone,
    # VALU with one scalar instruction after each, and scalar alone
    one = lambda k: res["%s@4w" % k]["cu_ipc"] / 4.0
    out["one_wave_valu_per_simd_clk"] = one("v_add_u32")
    out["one_wave_valu_per_simd_clk_with_salu"] = one("v_add_u32_with_s_mul_i32")
    out["one_wave_salu_per_simd_clk"] = one("s_mul_i32")
    return out


if __name__ == "__main__":
    r = measure()
    for k, v in r.items():
        if k == "summary":
            print(json.dumps(v, indent=1))
        elif isinstance(v, dict):
            print("%-32s %6.3f wave-instr/clk/CU  %6.1f lanes/CU/clk  %.3f GHz  %.3g lane-op/s" %
                  (k, v["cu_ipc"], v["lanes_per_cu_per_clk"], v["ghz"], v["lane_ops_per_s"]))
    if len(sys.argv) > 1:
        with open(sys.argv[1], "w") as f:
            json.dump(r, f, indent=1)
