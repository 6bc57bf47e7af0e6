"""Benchmark of the radiance-bucket lookup hot path on one MI355X.

Workload (default): the large configuration -- a 2048 x 2048 bucket matrix of
16 x 16 RGBA samples (smooth synthetic radiance, FP32 master copy, 17.2 GB)
stored as FP8 E4M3 with one FP32 scale per bucket, seen by 8 views of
3840 x 2160 pixels of a height field (66,355,200 fragments).  One step is one
pass of the whole hot path over that batch, as a fitting loop runs it:

    quantise   FP32 master texture -> FP8 storage            (rt_quantize)
    forward    per-fragment lookup from the FP8 texture      (rt_lookup_fwd)
    backward   dL/dtexture (dense, deterministic), dL/dview,
               dL/duv for i.i.d. N(0,1) upstream gradients   (rt_lookup_bwd)

The fragments are visited in the order of a visit plan (rt_plan_fragments:
the G-buffer sorted by bucket and cell), built once for the G-buffer before
the timed steps, as a fit whose cameras stay fixed builds it once; the
upstream gradient is in plan order.  The same step in image order (32 x 8
pixel tiles) and the step with the plan rebuilt every time are timed beside
it.  All inputs are resident in HBM before timing starts; the timed steps run
without the per-kernel event timer, which gets a separate pass of the same
steps (--graph: replays of the step captured in a HIP graph).  `value` is
fragments (lookups) per second of the whole step.  The JSON line also carries
the roofline of the dominant kernel (HIP events on the launch stream), the
hot path's kernels beside it, per-format forward numbers (FP32 / BF16 / FP8
storage), the FP64 CPU oracle timed on view 0, and the bake, minification,
shadow and dictionary measurements on the single-view workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--storage fp8]
                    [--order plan|image] [--no-cpu-baseline] [--no-extras] [--graph]
    python bench.py --save-inputs DIR      (write the inputs; then --load-inputs DIR)
    python bench.py --calibrate-copy       (plain copy kernel for the PMC scale)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the environment of the bake measurement: 8 spherical Gaussian lobes (axis
# xyz, sharpness, amplitude per channel) and an ambient term
BAKE_LOBES = [(0.3, -0.2, 1.0, 3.0, 0.8, 0.3, 0.1, 0.5), (1.0, 0.5, 0.4, 2.0, 0.1, 0.6, 0.2, 0.0),
              (-0.6, 0.9, 0.2, 1.5, 0.3, 0.1, 0.7, 0.9), (0.0, 0.0, 1.0, 8.0, 1.0, 1.0, 1.0, 0.0),
              (0.7, -0.7, 0.1, 4.0, 0.2, 0.0, 0.5, 0.1), (-0.2, -0.9, 0.4, 6.0, 0.0, 0.4, 0.3, 0.2),
              (0.5, 0.5, 0.7, 12.0, 0.6, 0.6, 0.0, 0.3), (-1.0, 0.1, 0.3, 1.0, 0.1, 0.2, 0.3, 0.4)]
BAKE_AMBIENT = (0.05, 0.05, 0.05, 0.0)

METRIC = "lookups/s + % HBM peak, fwd & bwd; FP32 vs BF16/FP8 texture at stated error"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# Source file of each kernel whose counters are committed under profiles/: a
# summary counts as current while its kernel's file and the shared headers
# (device helpers, launch constants) are unchanged.
KERNEL_SOURCES = {
    "k_lookup_fwd": "rt_lookup.hip", "k_lookup_lod": "rt_lookup.hip",
    "k_lookup_light": "rt_lookup.hip", "k_quant_bf16": "rt_quantize.hip",
    "k_quant_fp8": "rt_quantize.hip", "k_pack_bits_flat": "rt_quantize.hip",
    "k_bwd_fragment": "rt_backward.hip", "k_segacc": "rt_backward.hip",
    "k_segacc_big": "rt_backward.hip", "k_payload": "rt_backward.hip",
    "k_bake_env": "rt_bake.hip", "k_keys_in_order": "rt_backward.hip",
    "k_plan_keys": "rt_backward.hip", "k_plan_gather": "rt_backward.hip",
    "k_permute_rows": "rt_backward.hip",
    "k_bake_shadow": "rt_bake.hip", "k_build_mip": "rt_mip.hip",
    "k_vq_assign": "rt_dictionary.hip", "k_mip_adjoint": "rt_lod_backward.hip",
}
SHARED_SOURCES = ["rt_device.hpp", "rt_kernels.hpp"]
# kernels whose traffic depends on the order of the fragments: their counter
# summaries are kept per order (a "_plan" suffix for the planned step)
PLAN_SENSITIVE = {"k_lookup_fwd", "k_bwd_fragment", "k_segacc", "k_segacc_big"}

# the shadow measurement (Sec. 5, Shadowing): balls over the plane tile, a sun
# disc and a spherical lamp
SHADOW_BALLS = 16
SHADOW_CASES = (("sun", 1, "nearest"), ("sun", 16, "nearest"), ("sun", 64, "nearest"),
                ("lamp", 16, "bilinear"))

# the bucket-dictionary measurement: the matrix as repetitive buckets (each a
# noisy copy of one of DICT_PROTOTYPES buckets of the smooth texture), encoded
# into DICT_ENTRIES entries by DICT_ITERATIONS Lloyd steps
DICT_PROTOTYPES = 64
DICT_ENTRIES = 256
DICT_NOISE = 0.01
DICT_ITERATIONS = 3


def source_code(text: str) -> str:
    """C++ source without its comments and with whitespace collapsed: what a
    profile depends on (an edited comment leaves the kernels as they were)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(kernel: str) -> str:
    """Hash of the code (comments left out) of the sources that make up
    `kernel`: its file and the shared headers."""
    h = hashlib.sha256()
    for f in SHARED_SOURCES + [KERNEL_SOURCES[kernel]]:
        with open(os.path.join(ROOT, "paper_2301_01719_amd", "csrc", f)) as fh:
            h.update(source_code(fh.read()).encode())
    return h.hexdigest()[:16]


def pmc_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, or None when
    the summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if kernel not in KERNEL_SOURCES or vals.get("source_hash") != source_hash(kernel):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_shadow(rt, w, gb, reps, timed):
    """Shadowing on the workload's matrix and G-buffer: the bake of a 1-bit
    shadow texture from SHADOW_BALLS balls, the 1-bit packer on a one-channel
    FP32 matrix, and the light lookups of SHADOW_CASES.  With timed=False the
    kernels only run (for a profiler) and nothing is returned."""
    import numpy as np
    import torch
    from paper_2301_01719_amd import workloads as wl
    dev = gb.uv.device
    W, H, n = w.W, w.H, w.n
    N = gb.count
    nb = W * H
    wpb = rt.bit_words(n)
    balls = wl.shadow_balls(SHADOW_BALLS, seed=w.seed).numpy()
    origins = wl.bucket_origins(W, H, device=dev)
    words = torch.empty((H, W, wpb), dtype=torch.int32, device=dev)
    flags = (wl.uniform(w.seed, wl.S_TEXTURE, torch.arange(nb * n * n, device=dev)) < 0.5)
    x1 = flags.to(torch.float32).reshape(H, W, n, n, 1)
    del flags
    src = rt.Texture(x1, W, H, n, 1)
    packed = torch.empty_like(words)

    def light_of(kind, S):
        vec = (wl.sun_light(S) if kind == "sun" else wl.lamp_light(S)).numpy()
        return rt.make_light(vec, "directional" if kind == "sun" else "point")

    out = torch.empty((N, 1), dtype=torch.float32, device=dev)

    def everything():
        rt.bake_shadow(W, H, n, origins, balls, out=words)
        rt._check(rt.LIB.rt_quantize(src.handle, rt.RT_FMT_BIT1, rt._ptr(packed), None,
                                     rt._stream(dev)))
    stex = rt.Texture(words, W, H, n, 1, "bit1")
    if not timed:
        for _ in range(reps):
            everything()
            for kind, S, mode in SHADOW_CASES:
                rt.lookup_light(stex, gb.uv, gb.tbn, light_of(kind, S),
                                pos=gb.pos if kind == "lamp" else None, mode=mode, out=out,
                                image=gb.image)
        torch.cuda.synchronize()
        return None
    for _ in range(2):
        everything()
    torch.cuda.synchronize()
    rt.profile_reset()
    rt.profile_enable(True)
    for _ in range(reps):
        everything()
    torch.cuda.synchronize()
    rt.profile_enable(False)
    prof = rt.profile_read()
    bake_ms = prof["k_bake_shadow"][1] / prof["k_bake_shadow"][0]
    pack_ms = prof["k_pack_bits"][1] / prof["k_pack_bits"][0]
    pack_bytes = nb * n * n * 4 + nb * wpb * 4
    lit = float((torch.bitwise_and(
        words.reshape(-1, 1) >> torch.arange(32, device=dev, dtype=torch.int32)[None], 1)
        .sum()) / (nb * n * n))
    cases = {}
    for kind, S, mode in SHADOW_CASES:
        L = light_of(kind, S)
        pos = gb.pos if kind == "lamp" else None
        for _ in range(3):
            rt.lookup_light(stex, gb.uv, gb.tbn, L, pos=pos, mode=mode, out=out, image=gb.image)
        torch.cuda.synchronize()
        ms = []
        for _ in range(20):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            rt.lookup_light(stex, gb.uv, gb.tbn, L, pos=pos, mode=mode, out=out, image=gb.image)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        q = [round(float(v), 5) for v in np.percentile(np.array(ms), [10, 50, 90])]
        gbytes = N * (8 + 36 + 4 + (12 if pos is not None else 0))  # uv, frame, (pos), out
        cases[f"{kind}{S}_{mode}"] = {
            "light": kind, "samples": S, "mode": mode, "ms_p10_p50_p90": q,
            "fragments_per_s": round(N / (q[1] * 1e-3), 1),
            "fragment_samples_per_s": round(N * S / (q[1] * 1e-3), 1),
            "gbuffer_GBps": round(gbytes / (q[1] * 1e-3) / 1e9, 1),
            "gbuffer_hbm_frac": round(gbytes / (q[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "mean_visibility": round(float(out.mean()), 4)}
    del x1, src, packed
    return {"texture": f"{W}x{H} buckets of {n}x{n} bits ({nb * wpb * 4} bytes)",
            "bake_ms": round(bake_ms, 5), "bake_balls": SHADOW_BALLS,
            "bake_ray_ball_tests_per_s": round(nb * n * n * SHADOW_BALLS / (bake_ms * 1e-3), 1),
            "bake_lit_fraction": round(lit, 4),
            "pack_ms": round(pack_ms, 5), "pack_alg_bytes": pack_bytes,
            "pack_GBps": round(pack_bytes / (pack_ms * 1e-3) / 1e9, 1),
            "pack_hbm_frac": round(pack_bytes / (pack_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "light_lookups": cases,
            "note": "1-bit shadow texture baked from balls over the plane tile, read by the "
                    "G-buffer with a sun disc (directional samples, nearest bucket) and a "
                    "spherical lamp (point samples from each fragment's position, "
                    "bilinear-bucket); G-buffer bytes per fragment: uv 8, frame 36, "
                    "position 12 (lamp), out 4"}


def run_dictionary(rt, w, gb, tex32, reps, timed):
    """The bucket dictionary on the workload's matrix: a repetitive texture
    (every bucket a noisy copy of one of DICT_PROTOTYPES buckets of the smooth
    texture), DICT_ITERATIONS Lloyd steps into DICT_ENTRIES entries from
    seeded initial rows, then the lookup through the dictionary against the
    plain lookup of the repetitive texture.  timed=False only runs the
    kernels (for a profiler)."""
    import numpy as np
    import torch
    from paper_2301_01719_amd import workloads as wl
    dev = gb.uv.device
    W, H, n, C = w.W, w.H, w.n, w.C
    M, D, K = W * H, n * n * C, DICT_ENTRIES
    src = tex32.reshape(M, D)
    pick = (wl.uniform64(w.seed, wl.S_TEXTURE, torch.arange(DICT_PROTOTYPES, device=dev))
            * M).to(torch.int64)
    lab = (wl.uniform64(w.seed + 1, wl.S_TEXTURE, torch.arange(M, device=dev))
           * DICT_PROTOTYPES).to(torch.int64)
    X = src[pick][lab]
    a, b = wl.normal_pair(w.seed, wl.S_NOISE, M * D // 2, dev)
    X += DICT_NOISE * torch.cat([a, b]).reshape(M, D)
    del a, b, lab
    X = X.contiguous()
    init = (wl.uniform64(w.seed + 2, wl.S_TEXTURE, torch.arange(K, device=dev)) * M).to(torch.int64)
    cb = X[init].contiguous()
    ws = torch.empty(rt.LIB.rt_vq_update_workspace(M, D, K), dtype=torch.uint8, device=dev)
    out = torch.empty((gb.count, C), dtype=torch.float32, device=dev)

    def step():
        asg = rt.vq_assign(X, cb)
        rt.vq_update(X, asg, cb, workspace=ws)
        return asg
    if not timed:
        for _ in range(reps):
            asg = step()
        dtex = rt.DictionaryTexture(cb.reshape(K, n, n, C), asg.reshape(H, W), W, H, n, C)
        for _ in range(reps):
            rt.lookup_fwd(dtex, gb.uv, gb.tbn, gb.view, out=out, image=gb.image)
        torch.cuda.synchronize()
        return None
    rt.profile_reset()
    rt.profile_enable(True)
    for _ in range(DICT_ITERATIONS):
        asg = step()
    torch.cuda.synchronize()
    rt.profile_enable(False)
    prof = rt.profile_read()
    assign_ms = prof["k_vq_assign"][1] / prof["k_vq_assign"][0]
    upd = [k for k in ("k_vq_hist", "k_scan", "k_vq_scatter", "k_vq_pieces", "k_vq_combine")]
    update_ms = sum(prof[k][1] for k in upd) / DICT_ITERATIONS
    asg, dist = rt.vq_assign(X, cb, want_dist=True)
    torch.cuda.synchronize()
    flops = 2.0 * M * K * D
    idx8 = asg.to(torch.uint8).reshape(H, W)
    dtex = rt.DictionaryTexture(cb.reshape(K, n, n, C), idx8, W, H, n, C)
    ptex = rt.Texture(X.reshape(H, W, n, n, C), W, H, n, C)

    def timed_lookup(tex):
        for _ in range(3):
            rt.lookup_fwd(tex, gb.uv, gb.tbn, gb.view, out=out, image=gb.image)
        torch.cuda.synchronize()
        ms = []
        for _ in range(30):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rt.lookup_fwd(tex, gb.uv, gb.tbn, gb.view, out=out, image=gb.image)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return [round(float(v), 5) for v in np.percentile(np.array(ms), [10, 50, 90])]
    q_dict = timed_lookup(dtex)
    o_dict = out.clone()
    q_plain = timed_lookup(ptex)
    diff = (o_dict - out).abs()
    mse = float((diff.double() ** 2).mean())
    res = {"rows": M, "dim": D, "entries": K, "prototypes": DICT_PROTOTYPES, "noise": DICT_NOISE,
           "iterations": DICT_ITERATIONS,
           "assign_ms": round(assign_ms, 5),
           "assign_TFLOPs": round(flops / (assign_ms * 1e-3) / 1e12, 2),
           "assign_mfma_frac": round(flops / (assign_ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4),
           "update_ms": round(update_ms, 5),
           "lloyd_step_ms": round(assign_ms + update_ms, 5),
           "mean_sq_distance": round(float(dist.double().mean()), 6),
           "dictionary_bytes": K * D * 4 + M, "texture_bytes": M * D * 4,
           "lookup_ms_p10_p50_p90": q_dict, "plain_lookup_ms_p10_p50_p90": q_plain,
           "lookup_lookups_per_s": round(gb.count / (q_dict[1] * 1e-3), 1),
           "lookup_max_abs_diff_vs_plain": float(diff.max()),
           "lookup_psnr_db_vs_plain": round(10 * np.log10(1.0 / max(mse, 1e-30)), 2),
           "note": "FP32 entries, 1-byte entry numbers; the assignment is an M x K x D contraction "
                   "on v_mfma_f32_16x16x4_f32 (peak %.1f TFLOP/s)" % FP32_MFMA_PEAK_TFLOPS}
    del X, cb, ws, dtex, ptex
    return res


def calibrate_copy():
    import torch
    n = 1 << 28  # 1 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "calibrate_copy_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--storage", default="fp8", choices=["f32", "bf16", "fp8"])
    ap.add_argument("--order", default="plan", choices=["plan", "image"],
                    help="visit the fragments in plan order (the plan built once, before the "
                         "timed steps) or in image order (32x8 pixel tiles)")
    ap.add_argument("--extras-workload", default="c2",
                    help="workload of the bake, minification, shadow and dictionary measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the bake, minification, shadow and dictionary measurements")
    ap.add_argument("--no-formats", action="store_true",
                    help="skip the per-storage-format forward comparison")
    ap.add_argument("--no-multi-view", action="store_true",
                    help="skip the 64-view forward in plan and image order")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the step captured in a HIP graph (same kernels, no "
                         "host launch gaps)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--save-inputs", default=None, metavar="DIR",
                    help="generate the workload's inputs, write them to DIR and exit (so that a "
                         "profiled run can load them and launch no input-generating kernels)")
    ap.add_argument("--load-inputs", default=None, metavar="DIR",
                    help="read the inputs written by --save-inputs")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many steps (for rocprofv3) and print the line")
    ap.add_argument("--profile-plan", type=int, default=0,
                    help="with --profile-steps: also build the visit plan this many times")
    ap.add_argument("--profile-image-steps", type=int, default=0,
                    help="with --profile-steps: also run this many steps in image order")
    ap.add_argument("--profile-bake", type=int, default=0,
                    help="with --profile-steps: also run this many bakes of the matrix")
    ap.add_argument("--profile-mip", type=int, default=0,
                    help="with --profile-steps: also build the mip chain and run the "
                         "level-of-detail lookup this many times")
    ap.add_argument("--profile-dictionary", type=int, default=0,
                    help="with --profile-steps: also run this many Lloyd steps and dictionary "
                         "lookups")
    ap.add_argument("--profile-shadow", type=int, default=0,
                    help="with --profile-steps: also run the shadow bake, the 1-bit packer "
                         "and the light lookups this many times")
    return ap.parse_args()


INPUT_FILES = ("tex32", "uv", "tbn", "view", "grad_out")


def save_inputs(w, dev, path):
    """The workload's inputs as raw little-endian arrays plus a JSON index."""
    import numpy as np
    import torch
    from paper_2301_01719_amd import workloads as wl
    os.makedirs(path, exist_ok=True)
    tex32 = w.make_texture(dev)
    gb = w.make_gbuffer(dev)
    go = wl.grad_out(gb.count, w.C, seed=w.seed, device=dev)
    torch.cuda.synchronize()
    index = {"workload": w.name, "image": list(gb.image) if gb.image else None, "arrays": {}}
    for name, t in zip(INPUT_FILES, (tex32, gb.uv, gb.tbn, gb.view, go)):
        a = t.cpu().numpy()
        a.tofile(os.path.join(path, name + ".bin"))
        index["arrays"][name] = {"shape": list(a.shape), "dtype": str(a.dtype)}
        del a
    with open(os.path.join(path, "index.json"), "w") as fh:
        json.dump(index, fh)
    print(json.dumps({"saved_inputs": path, "workload": w.name}), flush=True)


def load_inputs(w, dev, path):
    """(tex32, GBuffer, grad_out) from a --save-inputs directory: host reads
    and copies to the device only, no kernels of the input generator."""
    import numpy as np
    import torch
    from paper_2301_01719_amd import workloads as wl
    with open(os.path.join(path, "index.json")) as fh:
        index = json.load(fh)
    if index["workload"] != w.name:
        raise SystemExit(f"{path} holds inputs of {index['workload']}, not {w.name}")
    out = {}
    for name in INPUT_FILES:
        meta = index["arrays"][name]
        a = np.fromfile(os.path.join(path, name + ".bin"), dtype=meta["dtype"])
        out[name] = torch.from_numpy(a.reshape(meta["shape"])).to(dev)
        del a
    gb = wl.GBuffer(out["uv"], out["tbn"], out["view"],
                    tuple(index["image"]) if index["image"] else None)
    return out["tex32"], gb, out["grad_out"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, tex32, gb, go, storage, N):
    """The FP64 oracle on one view of the workload, doing that view's share of
    the step: the quantiser over the view's share of the bucket matrix (the
    views split the step's work evenly), the forward and the backward of
    every fragment of the view (view and uv gradients), and the dense texel
    gradient of the view's share of the matrix (a window of whole bucket rows)
    written once in binary64.  The oracle reads the FP32 texture (its lookup
    costs the same for any storage format).  Timed single-threaded and on all
    host threads, median of 3 each."""
    import numpy as np
    import oracle
    W, H, n, C = w.W, w.H, w.n, w.C
    nv = (gb.image[1] * gb.image[2]) if gb.image else N
    uv_h, tbn_h, view_h = (t[:nv].cpu().numpy() for t in (gb.uv, gb.tbn, gb.view))
    go_h = go[:nv].cpu().numpy()
    nb = W * H
    rows_h = max(1, int(round(H * nv / N)))  # bucket rows of the view's share
    share = rows_h * W
    per = n * n * C
    tex_h = tex32.cpu().numpy()
    rows = tex_h.reshape(nb, per)[:share]
    otex = oracle.Tex(tex_h, W, H, n, C)
    full_threads = oracle.num_threads()
    fmt = {"bf16": oracle.FMT_BF16, "fp8": oracle.FMT_FP8_E4M3}.get(storage)

    def one_step():
        t0 = time.perf_counter()
        if fmt is not None:
            oracle.quantize(rows, share, per, fmt)
        t1 = time.perf_counter()
        oracle.lookup_fwd(otex, uv_h, tbn_h, view_h)
        t2 = time.perf_counter()
        r = oracle.lookup_bwd(otex, uv_h, tbn_h, view_h, go_h, window=(0, 0, W, rows_h),
                              want_abs=False)
        t3 = time.perf_counter()
        del r
        return t3 - t0, (t1 - t0, t2 - t1, t3 - t2)

    res = {}
    for label, threads in (("single_thread", 1), ("all_threads", full_threads)):
        oracle.set_num_threads(threads)
        runs = [one_step() for _ in range(3)]
        med = sorted(r[0] for r in runs)[1]
        parts = [float(np.median([r[1][k] for r in runs])) for k in range(3)]
        res[label] = {"threads": threads, "s_per_step": round(med, 3),
                      "lookups_per_s": round(nv / med, 1), "quantise_s": round(parts[0], 3),
                      "forward_s": round(parts[1], 3), "backward_s": round(parts[2], 3)}
    oracle.set_num_threads(full_threads)
    a = res["all_threads"]
    return {"value": a["lookups_per_s"], "unit": "lookups/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": (f"view 0 of the workload ({nv} of {N} fragments) with its share of the "
                       f"step: the {storage} quantiser over {share} of {nb} buckets, the forward "
                       f"and backward of every fragment of the view (view and uv gradients), and "
                       f"the dense texel gradient of bucket rows 0..{rows_h - 1} written once in "
                       f"binary64; median of 3 runs on all {a['threads']} host threads "
                       f"({a['s_per_step']} s per step) and of 3 single-threaded "
                       f"({res['single_thread']['s_per_step']} s)"),
            "single_thread_lookups_per_s": res["single_thread"]["lookups_per_s"],
            "runs": res, "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def timed_launches(fn, reps, cold_scratch=None):
    """Median and p10/p90 of `reps` launches of fn, each bracketed by HIP
    events on the current stream (the library launches on it)."""
    import numpy as np
    import torch
    ms = []
    for _ in range(reps):
        if cold_scratch is not None:
            cold_scratch.fill_(1.0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return [round(float(v), 5) for v in np.percentile(np.array(ms), [10, 50, 90])], ms


def run_multi_view(rt, dev):
    """The 64-view workload's forward (512 x 512 buckets of 16 x 16 RGBA, 64
    views of 1024 x 1024, one launch) per storage format, in plan order, in
    image order (32 x 8 pixel tiles) and in plan order with bucket tiles
    staged in LDS (RT_FWD_STAGE_BUCKETS), with its algorithmic bytes."""
    import torch
    from paper_2301_01719_amd import workloads as wl
    w = wl.WORKLOADS["c3"]
    W, H, n, C = w.W, w.H, w.n, w.C
    tex32 = w.make_texture(dev)
    gb = w.make_gbuffer(dev)
    N = gb.count
    master = rt.Texture(tex32, W, H, n, C)
    idx, _ = rt.debug_indices(master, gb.uv, gb.tbn, gb.view)
    x0 = torch.clamp(idx[:, 2], max=n - 2).to(torch.int64)
    y0 = torch.clamp(idx[:, 3], max=n - 2).to(torch.int64)
    b = idx[:, 1].to(torch.int64) * W + idx[:, 0].to(torch.int64)
    taps = torch.cat([b * n * n + (y0 + dy) * n + (x0 + dx) for dy in (0, 1) for dx in (0, 1)])
    uniq = int(torch.unique(taps).numel())
    ub = int(torch.unique(b).numel())
    del idx, x0, y0, b, taps
    order, puv, ptbn, pview = rt.plan_fragments(master, gb.uv, gb.tbn, gb.view, image=gb.image)
    out = torch.empty((N, C), dtype=torch.float32, device=dev)
    res = {"workload": w.name, "fragments": N, "unique_texels_touched": uniq}
    keep = []
    for fmt in ("f32", "bf16", "fp8"):
        tex = master
        if fmt != "f32":
            c_, s_ = rt.quantize(master, fmt)
            tex = rt.Texture(c_, W, H, n, C, fmt, s_)
            keep.append((c_, s_, tex))
        eb = {"f32": 4, "bf16": 2, "fp8": 1}[fmt]
        alg = N * 56 + N * C * 4 + uniq * C * eb + (ub * 4 if fmt == "fp8" else 0)
        r = {}
        for tag, args_ in (("plan", (puv, ptbn, pview, None, False)),
                           ("image", (gb.uv, gb.tbn, gb.view, gb.image, False)),
                           ("plan_staged_buckets", (puv, ptbn, pview, None, True))):
            u, t, v, im, st = args_
            fn = lambda: rt.lookup_fwd(tex, u, t, v, out=out, image=im, stage_buckets=st)
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            q, _ = timed_launches(fn, 20)
            r[tag] = {"fwd_ms_p10_p50_p90": q,
                      "fwd_lookups_per_s": round(N / (q[1] * 1e-3), 1),
                      "fwd_hbm_frac": round(alg / (q[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        r["alg_bytes"] = alg
        res[fmt] = r
    del keep, master, tex32, gb, order, puv, ptbn, pview, out
    torch.cuda.empty_cache()
    return res


def run_extras(rt, args, dev):
    """The bake, minification, shadow and dictionary measurements on their own
    workload (the single-view matrix by default)."""
    import numpy as np
    import torch
    from paper_2301_01719_amd import workloads as wl
    w = wl.WORKLOADS[args.extras_workload]
    W, H, n, C = w.W, w.H, w.n, w.C
    tex32 = w.make_texture(dev)
    gb = w.make_gbuffer(dev)
    N = gb.count
    E = W * H * n * n * C
    master = rt.Texture(tex32, W, H, n, C)
    out = torch.empty((N, C), dtype=torch.float32, device=dev)
    # ---- the bake (write side): the same matrix from an analytic environment
    dst = torch.empty_like(tex32)
    for _ in range(2):
        rt.bake_environment(W, H, n, C, BAKE_LOBES, BAKE_AMBIENT, out=dst)
    torch.cuda.synchronize()
    rt.profile_reset()
    rt.profile_enable(True)
    reps = 10
    for _ in range(reps):
        rt.bake_environment(W, H, n, C, BAKE_LOBES, BAKE_AMBIENT, out=dst)
    torch.cuda.synchronize()
    rt.profile_enable(False)
    launches, total = rt.profile_read()["k_bake_env"]
    avg = total / launches
    bake = {"workload": w.name, "kernel": "k_bake_env", "avg_ms": round(avg, 5),
            "lobes": len(BAKE_LOBES), "texels_per_s": round(W * H * n * n / (avg * 1e-3), 1),
            "alg_bytes": E * 4, "GBps": round(E * 4 / (avg * 1e-3) / 1e9, 1),
            "hbm_frac": round(E * 4 / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "FP32 bake of the whole bucket matrix from 8 spherical Gaussian lobes along "
                    "every sample's reflection vector (Eqs. 4a, 4b), identity frames"}
    del dst
    # ---- minification: the mip chain and the level-of-detail lookup
    mip = None
    pow2 = lambda v: v > 0 and (v & (v - 1)) == 0
    if gb.duv is not None and pow2(W) and pow2(H):
        chain = rt.build_mips(master)
        L = len(chain)
        torch.cuda.synchronize()
        rt.profile_reset()
        rt.profile_enable(True)
        for _ in range(5):
            for l in range(1, L):
                rt.build_mip(chain[l - 1], out=chain[l].data)
        torch.cuda.synchronize()
        rt.profile_enable(False)
        build_ms = rt.profile_read()["k_build_mip"][1] / 5
        lvl_bytes = [t.W * t.H * n * n * C * 4 for t in chain]
        build_bytes = sum(lvl_bytes[:-1]) + sum(lvl_bytes[1:])
        lod = lambda: rt.lookup_fwd_lod(chain, gb.uv, gb.tbn, gb.view, gb.duv, out=out,
                                        image=gb.image)
        for _ in range(3):
            lod()
        torch.cuda.synchronize()
        q, _ = timed_launches(lod, 30)
        go_lod = torch.randn(out.shape, generator=torch.Generator(device=dev).manual_seed(17),
                             device=dev)
        ws_lod = torch.empty(max(rt.lookup_lod_bwd_workspace(chain, N), 1), dtype=torch.uint8,
                             device=dev)
        lodb = lambda: rt.lookup_lod_bwd(chain, gb.uv, gb.tbn, gb.view, gb.duv, go_lod,
                                         workspace=ws_lod, image=gb.image)
        for _ in range(2):
            lodb()
        torch.cuda.synchronize()
        bq, _ = timed_launches(lodb, 10)
        gls = [torch.zeros_like(t.data) for t in chain]
        torch.cuda.synchronize()
        rt.profile_reset()
        rt.profile_enable(True)
        for _ in range(3):
            for l in range(L - 1, 0, -1):
                rt.build_mip_adjoint(chain[l - 1], gls[l], gls[l - 1])
        torch.cuda.synchronize()
        rt.profile_enable(False)
        adj_ms = rt.profile_read()["k_mip_adjoint"][1] / 3
        adj_bytes = sum(lvl_bytes[1:]) + 2 * sum(lvl_bytes[:-1])
        mip = {"workload": w.name, "levels": L, "build_chain_ms": round(build_ms, 5),
               "build_alg_bytes": build_bytes,
               "build_hbm_frac": round(build_bytes / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "lod_fwd_ms_p10_p50_p90": q, "lod_fwd_lookups_per_s": round(N / (q[1] * 1e-3), 1),
               "lod_bwd_ms_p10_p50_p90": bq, "adjoint_chain_ms": round(adj_ms, 5),
               "adjoint_hbm_frac": round(adj_bytes / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del chain, gls, ws_lod, go_lod
    shadow = run_shadow(rt, w, gb, 5, timed=True) if gb.pos is not None else None
    dictionary = run_dictionary(rt, w, gb, tex32, 3, timed=True)
    return {"bake": bake, "mip": mip, "shadow": shadow, "dictionary": dictionary}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the lookup needs no communication between GPUs "
              "and the library runs on a single MI355X; sharding over several GPUs is not "
              "built. Use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import numpy as np
    import torch

    from paper_2301_01719_amd import workloads as wl

    dev = "cuda:0"
    w = wl.WORKLOADS[args.workload]
    if args.save_inputs:
        save_inputs(w, dev, args.save_inputs)
        return

    from paper_2301_01719_amd import radtex as rt

    W, H, n, C = w.W, w.H, w.n, w.C
    t_setup = time.time()
    if args.load_inputs:
        tex32, gb, go = load_inputs(w, dev, args.load_inputs)
    else:
        tex32 = w.make_texture(dev)
        gb = w.make_gbuffer(dev)
        go = wl.grad_out(gb.count, C, seed=w.seed, device=dev)
    N = gb.count
    torch.cuda.synchronize()
    print(f"# inputs ready in {time.time() - t_setup:.1f} s: {W}x{H} buckets of {n}x{n}x{C}, "
          f"{N} fragments", file=sys.stderr, flush=True)

    master = rt.Texture(tex32, W, H, n, C)
    E = W * H * n * n * C
    storage = {}
    if args.storage != "f32":
        codes, scales = rt.quantize(master, args.storage)
        storage["tex"] = rt.Texture(codes, W, H, n, C, args.storage, scales)
        storage["codes"], storage["scales"] = codes, scales
    else:
        storage["tex"] = master
    tex_s = storage["tex"]
    grad_tex = torch.empty((H, W, n, n, C), dtype=torch.float32, device=dev)
    ws = torch.empty(rt.bwd_workspace_bytes(tex_s, N), dtype=torch.uint8, device=dev)
    out = torch.empty((N, C), dtype=torch.float32, device=dev)

    # the visit plan, built once for the G-buffer (its rebuild is timed below)
    pws = torch.empty(max(rt.plan_workspace_bytes(tex_s, N), 256), dtype=torch.uint8, device=dev)
    pbuf = (torch.empty(N, dtype=torch.int32, device=dev),
            torch.empty((N, 2), dtype=torch.float32, device=dev),
            torch.empty((N, 3, 3), dtype=torch.float32, device=dev),
            torch.empty((N, 3), dtype=torch.float32, device=dev))

    def build_plan():
        rt.plan_fragments(tex_s, gb.uv, gb.tbn, gb.view, image=gb.image, workspace=pws,
                          out=pbuf)

    build_plan()
    order, puv, ptbn, pview = pbuf
    pgo = rt.plan_permute(order, go)  # the upstream gradient in plan order
    torch.cuda.synchronize()

    def quantise():
        if args.storage != "f32":
            rt._check(rt.LIB.rt_quantize(master.handle, rt.FORMATS[args.storage],
                                         rt._ptr(storage["codes"]), rt._ptr(storage["scales"]),
                                         rt._stream(dev)))

    def step_plan():
        quantise()
        rt.lookup_fwd(tex_s, puv, ptbn, pview, out=out)
        rt.lookup_bwd(tex_s, puv, ptbn, pview, pgo, workspace=ws, grad_tex=grad_tex)

    def step_image():
        quantise()
        rt.lookup_fwd(tex_s, gb.uv, gb.tbn, gb.view, out=out, image=gb.image)
        rt.lookup_bwd(tex_s, gb.uv, gb.tbn, gb.view, go, workspace=ws, grad_tex=grad_tex,
                      image=gb.image)

    def step_rebuilt():
        build_plan()
        rt.plan_permute(order, go, out=pgo)  # the upstream gradient into plan order
        step_plan()

    planned = args.order == "plan"
    step = step_plan if planned else step_image

    if args.profile_steps:
        for _ in range(args.profile_steps):
            step()
        for _ in range(args.profile_plan):
            build_plan()
        for _ in range(args.profile_image_steps):
            step_image()
        torch.cuda.synchronize()
        if args.profile_bake or args.profile_mip or args.profile_shadow or args.profile_dictionary:
            profile_extras(rt, args, dev)
        print(json.dumps({"profile_steps": args.profile_steps, "workload": w.name,
                          "order": args.order}), flush=True)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    run = step
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        torch.cuda.synchronize()
        run = graph.replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = N / (ms_per_step * 1e-3)

    # the other two orders of the same step, fewer repetitions
    def wall(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / reps
    reps = max(3, args.steps // 4)
    other = {"plan_ms_per_step": round(ms_per_step if planned else wall(step_plan, reps), 5),
             "image_order_ms_per_step": round(wall(step_image, reps) if planned
                                              else ms_per_step, 5),
             "plan_rebuilt_ms_per_step": round(wall(step_rebuilt, reps), 5)}
    plan_ms, _ = timed_launches(build_plan, 5)
    other["plan_build_ms_p10_p50_p90"] = plan_ms

    # per-kernel durations: the same number of steps launched eagerly, each
    # kernel bracketed by HIP events on its launch stream
    def kernel_ms(fn, reps):
        rt.profile_reset()
        rt.profile_enable(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        rt.profile_enable(False)
        return rt.profile_read()
    prof = kernel_ms(step, args.steps)
    prof_img = kernel_ms(step_image if planned else step_plan, 5)

    # ---- algorithmic bytes per launch of each kernel ------------------------
    eb = {"f32": 4, "bf16": 2, "fp8": 1}[args.storage]
    idx, _ = rt.debug_indices(tex_s, gb.uv, gb.tbn, gb.view)
    x0 = torch.clamp(idx[:, 2], max=n - 2).to(torch.int64)
    y0 = torch.clamp(idx[:, 3], max=n - 2).to(torch.int64)
    b = idx[:, 1].to(torch.int64) * W + idx[:, 0].to(torch.int64)
    taps = torch.cat([b * n * n + (y0 + dy) * n + (x0 + dx) for dy in (0, 1) for dx in (0, 1)])
    uniq_texels = int(torch.unique(taps).numel())
    uniq_buckets = int(torch.unique(b).numel())
    # the 128-byte lines those taps lie in, per storage format (texel t of the
    # bucket-major array starts at byte t C eb): what a line-granular memory
    # system fetches at least
    uniq_lines = {f: int(torch.unique(taps * (C * e) // 128).numel())
                  for f, e in (("f32", 4), ("bf16", 2), ("fp8", 1))}
    cnt = torch.bincount(b, minlength=W * H)
    small = cnt <= 64
    big = (cnt > 64) & (cnt <= 2048)
    n_small, n_big = int(small.sum()), int(big.sum())
    r_small, r_big = int(cnt[small].sum()), int(cnt[big].sum())
    del taps, idx, cnt, small, big, x0, y0, b
    texel_bytes = uniq_texels * C * eb + (uniq_buckets * 4 if args.storage == "fp8" else 0)
    gbuf = N * 56
    pay = N <= 64 * W * H and not planned
    rec = (4 + 8 + C * 4) if (pay or planned) else (4 + 4 + 8 + C * 4)
    alg = {
        "k_quant_bf16": E * 4 + E * 2,
        "k_quant_fp8": E * 4 + E + W * H * 4,
        "k_lookup_fwd": gbuf + N * C * 4 + texel_bytes,
        "k_bwd_fragment": gbuf + N * C * 4 + texel_bytes + N * (12 + 8) + N * (4 + 8),
        # tiles written + records read (in plan order or from the sorted
        # payload: key, fractions, upstream gradient; else also the record
        # number) + bucket ranges read (+ the list entries of the big pass)
        "k_segacc": n_small * n * n * C * 4 + r_small * rec + W * H * 8,
        "k_segacc_big": n_big * n * n * C * 4 + r_big * (4 + 4 + 8 + C * 4) + n_big * (8 + 4),
        "k_keys_in_order": N * 4,
        "k_plan_keys": gbuf + N * 4,
        "k_plan_gather": gbuf * 2 + N * 4 * 2,
    }
    if pay:
        alg["k_payload"] = N * 4 + W * H * 8 + r_small * (4 + 8 + C * 4 + 8 + C * 4)
    if n_big == 0:
        del alg["k_segacc_big"]

    def kernel_table(p, reps, with_alg=True):
        tab = {}
        for name, (launches, total) in p.items():
            if launches == 0:
                continue
            avg = total / launches
            entry = {"launches_per_step": launches / reps, "avg_ms": round(avg, 5),
                     "ms_per_step": round(total / reps, 5)}
            if with_alg and name in alg:
                entry["alg_bytes"] = alg[name]
                entry["GBps"] = round(alg[name] / (avg * 1e-3) / 1e9, 1)
                entry["hbm_frac"] = round(entry["GBps"] / HBM_PEAK_GBS, 4)
            tab[name] = entry
        return tab
    per_kernel = kernel_table(prof, args.steps)
    dom = max((k for k in per_kernel if k in alg), key=lambda k: per_kernel[k]["ms_per_step"])
    d = per_kernel[dom]
    wtag = args.workload + ("_plan" if planned and dom in PLAN_SENSITIVE else "")
    traffic = pmc_traffic(dom, wtag)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": d["hbm_frac"], "traffic": traffic,
                "alg_bytes_per_launch": d["alg_bytes"], "avg_ms": d["avg_ms"]}
    # the lookup's own kernels beside the dominant one
    hot_path = {}
    for k in ("k_lookup_fwd", "k_bwd_fragment", "k_segacc", "k_quant_fp8", "k_quant_bf16"):
        if k in per_kernel and "hbm_frac" in per_kernel[k]:
            e = per_kernel[k]
            hot_path[k] = {"avg_ms": e["avg_ms"], "GBps": e["GBps"], "hbm_frac": e["hbm_frac"],
                           "traffic": pmc_traffic(k, args.workload + (
                               "_plan" if planned and k in PLAN_SENSITIVE else ""))}

    # ---- forward per storage format (FP32 / BF16 / FP8) ----------------------
    formats = {}
    if not args.no_formats:
        fmts = ("f32", "bf16", "fp8")
        texs, keep = {"f32": master}, []
        for fmt in fmts[1:]:
            if fmt == args.storage:
                texs[fmt] = tex_s
                continue
            c_, s_ = rt.quantize(master, fmt)
            texs[fmt] = rt.Texture(c_, W, H, n, C, fmt, s_)
            keep.append((c_, s_))
        fu, ft, fv = (puv, ptbn, pview) if planned else (gb.uv, gb.tbn, gb.view)
        fimg = None if planned else gb.image
        outs = {fmt: torch.empty_like(out) for fmt in fmts}
        for fmt in fmts:
            for _ in range(3):
                rt.lookup_fwd(texs[fmt], fu, ft, fv, out=outs[fmt], image=fimg)
        torch.cuda.synchronize()
        scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        runs = {fmt: {False: [], True: []} for fmt in fmts}
        for cold, rounds in ((False, 40), (True, 15)):
            for r in range(rounds):
                for q in range(3):
                    fmt = fmts[(r + q) % 3]
                    _, ms = timed_launches(lambda: rt.lookup_fwd(texs[fmt], fu, ft, fv,
                                                                 out=outs[fmt], image=fimg),
                                           1, scratch if cold else None)
                    runs[fmt][cold].append(ms[0])
        pct = lambda v: [round(float(x), 5) for x in np.percentile(np.array(v), [10, 50, 90])]
        for fmt in fmts:
            warm, cold = pct(runs[fmt][False]), pct(runs[fmt][True])
            ebf = {"f32": 4, "bf16": 2, "fp8": 1}[fmt]
            fb = gbuf + N * C * 4 + uniq_texels * C * ebf + (uniq_buckets * 4 if fmt == "fp8"
                                                              else 0)
            e2e = (outs[fmt] - outs["f32"]).abs()
            lines = gbuf + N * C * 4 + uniq_lines[fmt] * 128 + (uniq_buckets * 4 if fmt == "fp8"
                                                                 else 0)
            formats[fmt] = {"fwd_ms_p10_p50_p90": warm, "fwd_ms_cold_p10_p50_p90": cold,
                            "fwd_line_floor_ms": round(lines / HBM_PEAK_GBS / 1e6, 5),
                            "fwd_lines_touched": uniq_lines[fmt],
                            "fwd_lookups_per_s": round(N / (warm[1] * 1e-3), 1),
                            "fwd_alg_GBps": round(fb / (warm[1] * 1e-3) / 1e9, 1),
                            "fwd_hbm_frac": round(fb / (warm[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "max_abs_diff_vs_f32_storage": float(e2e.max()),
                            "mean_abs_diff_vs_f32_storage": float(e2e.mean())}
            del e2e
            # the same launch with bucket tiles staged in LDS
            # (RT_FWD_STAGE_BUCKETS), bits compared with the plain launch's
            st_out = torch.empty_like(out)
            sfn = lambda: rt.lookup_fwd(texs[fmt], fu, ft, fv, out=st_out, image=fimg,
                                        stage_buckets=True)
            for _ in range(3):
                sfn()
            torch.cuda.synchronize()
            sq, _ = timed_launches(sfn, 20)
            formats[fmt]["staged_buckets_fwd_ms_p10_p50_p90"] = sq
            formats[fmt]["staged_buckets_bitwise_equal"] = bool(torch.equal(st_out, outs[fmt]))
            del st_out
        from scipy.stats import mannwhitneyu
        for fmt in ("bf16", "fp8"):
            for cold, tag in ((False, ""), (True, "_cold")):
                p = float(mannwhitneyu(runs[fmt][cold], runs["f32"][cold],
                                       alternative="less").pvalue)
                key = "fwd_ms_cold_p10_p50_p90" if cold else "fwd_ms_p10_p50_p90"
                formats[fmt]["faster_than_f32_p" + tag] = p
                formats[fmt]["faster_than_f32" + tag] = bool(p < 1e-3)
                formats[fmt]["band_below_f32" + tag] = bool(formats[fmt][key][2] <
                                                            formats["f32"][key][0])
        del scratch, texs, outs, keep

    # ---- the 64-view FP32 forward, plan order against image order -----------
    multi = None
    if not args.no_multi_view and args.workload != "c3":
        multi = run_multi_view(rt, dev)

    # ---- the FP64 oracle on a bounded sample (CPU baseline) ------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, tex32, gb, go, args.storage, N)

    extras = {}
    if not args.no_extras:
        del ws, grad_tex
        torch.cuda.empty_cache()
        extras = run_extras(rt, args, dev)

    order_desc = ("visit plan: the G-buffer ordered by bucket and cell once (rt_plan_fragments, "
                  "outside the timed steps), every per-fragment array in plan order"
                  if planned else
                  ("%dx%dx%d images visited in 32x8 pixel tiles" % gb.image if gb.image
                   else "flat"))
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "lookups/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "buckets": [W, H], "n": n, "channels": C,
                   "fragments": N, "storage": args.storage,
                   "step": "quantize(f32->%s) + forward + backward(grad_tex dense, grad_view, "
                           "grad_uv)" % args.storage, "mode": "nearest",
                   "fragment_order": order_desc,
                   "launch": "HIP graph replay" if args.graph else "eager"},
        "roofline": roofline,
        "hot_path": hot_path,
        "other_orders": other,
        "cpu_baseline": cpu,
        "kernels": per_kernel,
        "kernels_other_order": kernel_table(prof_img, 5, with_alg=False),
        "formats": formats,
        "multi_view_fwd": multi,
        "unique_texels_touched": uniq_texels,
        "source_hash": {k: source_hash(k) for k in sorted(KERNEL_SOURCES)},
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


def profile_extras(rt, args, dev):
    """The extras' kernels on their workload, for a profiler (nothing timed)."""
    import torch
    from paper_2301_01719_amd import workloads as wl
    w = wl.WORKLOADS[args.extras_workload]
    W, H, n, C = w.W, w.H, w.n, w.C
    tex32 = w.make_texture(dev)
    gb = w.make_gbuffer(dev)
    master = rt.Texture(tex32, W, H, n, C)
    out = torch.empty((gb.count, C), dtype=torch.float32, device=dev)
    if args.profile_bake:
        dst = torch.empty_like(tex32)
        for _ in range(args.profile_bake):
            rt.bake_environment(W, H, n, C, BAKE_LOBES, BAKE_AMBIENT, out=dst)
        del dst
    if args.profile_mip and gb.duv is not None:
        chain = rt.build_mips(master)
        for _ in range(args.profile_mip):
            for l in range(1, len(chain)):
                rt.build_mip(chain[l - 1], out=chain[l].data)
            rt.lookup_fwd_lod(chain, gb.uv, gb.tbn, gb.view, gb.duv, out=out, image=gb.image)
        gls = [torch.zeros_like(t.data) for t in chain]
        for _ in range(args.profile_mip):
            for l in range(len(chain) - 1, 0, -1):
                rt.build_mip_adjoint(chain[l - 1], gls[l], gls[l - 1])
        del chain, gls
    if args.profile_shadow and gb.pos is not None:
        run_shadow(rt, w, gb, args.profile_shadow, timed=False)
    if args.profile_dictionary:
        run_dictionary(rt, w, gb, tex32, args.profile_dictionary, timed=False)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
