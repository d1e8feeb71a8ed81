"""Build libbesselk.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); the host pass prints a
harmless warning that it does not know the feature.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbesselk.so")
RATES_LIB = os.path.join(HERE, "libvalurates.so")
SOURCES = ["bk_kernels.hip", "bk_mlp.hip", "bk_mle.hip"]
# rocSOLVER (Cholesky, triangular solves, inverse) and the rocBLAS handle it runs on
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas"]
ARCH = os.environ.get("BK_OFFLOAD_ARCH", "gfx950")


# Issue cost of a wave64 VALU instruction on gfx950 in CU clocks (one CU issues
# one full-rate wave64 VALU instruction per clock across its four SIMDs), measured
# on MI355X with independent chains of one instruction at a time: FP32 add, mul,
# fma, 32-bit integer add and moves run at about two per clock; FP32
# transcendentals at one per two clocks; FP64 reciprocal, square root and
# reciprocal square root at one per four; everything else checked (FP64 add, mul,
# fma, ldexp, rounding, conversions, FP32 max, ldexp and rounding, selects) at one
# per clock.
HALF_COST = ("v_add_f32", "v_sub_f32", "v_subrev_f32", "v_mul_f32", "v_fma_f32", "v_fmac_f32", "v_fmamk_f32",
             "v_fmaak_f32", "v_mac_f32", "v_add_u32", "v_sub_u32", "v_subrev_u32", "v_mov_b32")
DOUBLE_COST = ("v_exp_f32", "v_log_f32", "v_rcp_f32", "v_rsq_f32", "v_sqrt_f32", "v_sin_f32", "v_cos_f32",
               "v_rcp_iflag_f32", "v_exp_f16", "v_log_f16")
QUAD_COST = ("v_rcp_f64", "v_rsq_f64", "v_sqrt_f64")


def issue_cost(op):
    base = op.split("_e32")[0].split("_e64")[0].split("_dpp")[0].split("_sdwa")[0]
    if base in QUAD_COST:
        return 4.0
    if base in DOUBLE_COST:
        return 2.0
    if base in HALF_COST:
        return 0.5
    return 1.0


def _loops(lines):
    """(start, end) line spans of the loops of one function: a label and the last
    later branch back to it (a loop whose body has several paths has several back
    edges; the span covers them all)."""
    import re
    labels = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            labels[m.group(1)] = i
    last = {}
    for i, l in enumerate(lines):
        m = re.search(r"s_cbranch_\w+\s+(\.LBB\d+_\d+)|s_branch\s+(\.LBB\d+_\d+)", l)
        if m:
            lab = m.group(1) or m.group(2)
            if lab in labels and labels[lab] < i:
                last[lab] = i
    return [(labels[lab], i) for lab, i in last.items()]


def node_slots(asm_path):
    """VALU issue cost of one trapezoid node per K_nu kernel, in CU clocks per wave
    (issue_cost above), read from the gfx950 assembly of this build: the node loop
    is the innermost loop that evaluates the node exponential (v_exp_f32 for the
    FP32-term forms; the inlined FP64 exp, one v_ldexp_f64 without divisions or
    logarithms, for the plain form), and its cost is divided by the exponentials
    one trip evaluates (the plain form's paired walk evaluates two nodes a trip
    when both sides of the reference node are live)."""
    text = open(asm_path).read().split("\n")
    funcs = {}
    cur = None
    for l in text:
        if l and not l.startswith((" ", "\t", ".", ";")) and l.endswith(":") or (l.startswith("_Z") and ": ;" in l):
            cur = l.split(":")[0]
            funcs[cur] = []
        elif cur is not None:
            funcs[cur].append(l)
    want = {"plain": "k_besselkILi0", "mixed": "k_besselkILi1", "learned": "k_besselk_learnedILb1",
            # Matern kernels without statistics: FP64 output for plain, FP32 for the others
            "matern_plain": "k_maternILi0EdLb0", "matern_mixed": "k_maternILi1EfLb0",
            "matern_learned": "k_matern_learnedIfLb0"}
    out = {}
    for form, key in want.items():
        name = next((f for f in funcs if key in f), None)
        if name is None:
            continue
        body = funcs[name]
        best = None
        for a, b in _loops(body):
            seg = [x.strip() for x in body[a:b + 1]]
            ops = [x.split()[0] for x in seg if x.startswith("v_")]
            if form in ("plain", "matern_plain"):
                ok = ops.count("v_ldexp_f64") >= 1 and "v_div_scale_f64" not in ops and "v_frexp_mant_f64_e32" not in ops
            else:
                ok = any(o.startswith("v_exp_f32") for o in ops) and "v_div_scale_f64" not in ops
            if ok:
                slots = sum(issue_cost(o) for o in ops if not o.startswith("v_mfma"))
                # an unrolled loop evaluates several nodes per trip: one node exponential each
                per_trip = (ops.count("v_ldexp_f64") if form in ("plain", "matern_plain")
                            else sum(o.startswith("v_exp_f32") for o in ops))
                slots = slots / max(1, per_trip)
                if best is None or (b - a) < best[0]:
                    best = (b - a, slots)
        if best is not None:
            out[form] = best[1]
    return out


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-Wall", "-Wno-unused-function"]
    objs = []
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, s + ".o")
        cmd = [hipcc] + flags + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE), s))
        objs.append(obj)
    failed = False
    for p, s in procs:
        out, err = p.communicate()
        msg = "\n".join(l for l in err.decode().splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write("hipcc failed on %s:\n%s\n" % (s, msg))
        elif verbose and msg.strip():
            sys.stderr.write(msg + "\n")
    if failed:
        raise RuntimeError("HIP build failed")
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    # instruction-rate probe behind issue_cost (bench.py --workload valu-rates); its own
    # library, not part of the K_nu path
    cmd = [hipcc] + flags + ["-shared", "-o", RATES_LIB + ".tmp", os.path.join(CSRC, "valu_rates.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    if p.returncode != 0:
        raise RuntimeError("HIP build of valu_rates.hip failed:\n" + p.stderr.decode())
    os.replace(RATES_LIB + ".tmp", RATES_LIB)
    # node-loop issue slots of this build, for the benchmark's roofline accounting
    try:
        import json
        slots = {}
        for src in SOURCES[:2]:
            asm = os.path.join(CSRC, src + ".s")
            subprocess.check_call([hipcc] + flags + ["--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", asm],
                                  stderr=subprocess.DEVNULL)
            slots.update(node_slots(asm))
            os.remove(asm)
        with open(os.path.join(HERE, "node_slots.json"), "w") as f:
            json.dump(slots, f)
        if verbose:
            print("node-loop issue slots:", slots, flush=True)
    except Exception as e:  # the library is built; the slot table is an aid only
        sys.stderr.write("node-slot count skipped: %s\n" % e)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
