#!/usr/bin/env python3
"""Writes asm_steps.h: one K block of the pair GEMM (step 3 of the emulated
GEMM: every kept slice pair (s, t), s + t < G, multiplied on the int8 matrix
cores into the accumulator of its diagonal) as a single inline-asm block per
(S, G), for waves that own one 32 x 32 output block, and for G = 7, 8 one
per (S, G) for waves that own two blocks stacked in M.

The block runs the MFMAs of the current K block slice-major (A slice s with
every B slice it meets, highest first) and reads the next block's fragments
from LDS into the same registers as soon as their last MFMA of this block
has issued: A slice s after its group, B slice t after its last partner.
It ends by waiting for those reads, so every register it writes is complete
when it returns.  Keeping the reads inside the block keeps them out of the
compiler's view of LDS accesses: it then never orders them behind the
direct-to-LDS loads of later blocks, which may stay in flight.

Run from anywhere: python3 gen_asm_steps.py (writes asm_steps.h next to it).
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read(kind, j):
    return "ds_read_b128 %%[%s%d], %%[p%s] offset:%%[o%s%d]" % (kind, j, kind, kind, j)


NSPARE = 4


def step_lines(S, G):
    """The in-place order: each fragment register is refilled right after its
    last MFMA of the block.  The last NSPARE refills of that order would leave
    the final wait exposed, so those fragments go to spare registers instead,
    read early in the block (the caller moves them into place afterwards)."""
    T = min(S, G)
    last_s = {t: min(T - 1, G - 1 - t) for t in range(T)}
    seq = []  # ("m", s, t) or ("r", kind, j)
    for s in range(T):
        for t in range(T - 1, -1, -1):
            if s + t >= G:
                continue
            seq.append(("m", s, t))
            if last_s[t] == s:
                seq.append(("r", "b", t))
        seq.append(("r", "a", s))
    reads = [x for x in seq if x[0] == "r"]
    ns = min(NSPARE, len(reads) - 1)
    spare = reads[len(reads) - ns:]
    seq = [x for x in seq if x not in spare]
    lines = ["s_nop 4"]
    mfmas = 0
    pending = list(enumerate(spare))
    for x in seq:
        if x[0] == "m":
            _, s, t = x
            lines.append("v_mfma_i32_32x32x32_i8 %%[c%d], %%[a%d], %%[b%d], %%[c%d]" % (s + t, s, t, s + t))
            mfmas += 1
            # a spare read after each of the first MFMAs
            if pending:
                k, (_, kind, j) = pending.pop(0)
                lines.append("ds_read_b128 %%[x%d], %%[p%s] offset:%%[o%s%d]" % (k, kind, kind, j))
        else:
            lines.append(read(x[1], x[2]))
    for k, (_, kind, j) in pending:
        lines.append("ds_read_b128 %%[x%d], %%[p%s] offset:%%[o%s%d]" % (k, kind, kind, j))
    lines.append("s_waitcnt lgkmcnt(0)")
    return lines, T, [(kind, j) for (_, kind, j) in spare]


def spec(S, G):
    lines, T, spare = step_lines(S, G)
    text = "".join('            "%s\\n\\t"\n' % l for l in lines).rstrip("\n")
    frag = ["[a%d] \"+v\"(f.a[%d][0])" % (s, s) for s in range(T)] + ["[b%d] \"+v\"(f.b[%d][0])" % (t, t) for t in range(T)]
    outs = ["[c%d] \"+v\"(acc[%d][0][0])" % (g, g) for g in range(G)] + frag
    outs += ["[x%d] \"=&v\"(x[%d])" % (k, k) for k in range(len(spare))]
    moves = "".join("        f.%s[%d][0] = x[%d];\n" % (kind, j, k) for k, (kind, j) in enumerate(spare))
    addr = ['[pa] "v"(pa)', '[pb] "v"(pb)']
    addr += ["[oa%d] \"i\"(%d * OA)" % (s, s) for s in range(T)]
    addr += ["[ob%d] \"i\"(%d * OB)" % (t, t) for t in range(T)]
    rlines = [read("a", s) for s in range(T)] + [read("b", t) for t in range(T)] + ["s_waitcnt lgkmcnt(0)"]
    rtext = "".join('            "%s\\n\\t"\n' % l for l in rlines).rstrip("\n")
    rfrag = [x.replace('"+v"', '"=v"') for x in frag]
    j = ",\n              ".join
    return """template <>
struct AsmStep<%d, %d> {
    static constexpr bool available = true;
    template <int OA, int OB, typename F>
    __device__ __forceinline__ static void run(v16i (&acc)[%d][1][1], F &f, unsigned pa, unsigned pb) {
        v4i x[%d];
        asm volatile(
%s
            : %s
            : %s
            : "memory");
%s    }
    // the fragments of one block only (the first block of a term)
    template <int OA, int OB, typename F>
    __device__ __forceinline__ static void read(F &f, unsigned pa, unsigned pb) {
        asm volatile(
%s
            : %s
            : %s
            : "memory");
    }
};
""" % (S, G, G, max(len(spare), 1), text, j(outs), j(addr), moves, rtext, j(rfrag), j(addr))


def step_lines2(S, G):
    """As step_lines for a wave owning two 32 x 32 blocks stacked in M (two
    A fragments per slice, one B fragment): each kept pair's MFMA for both
    blocks in turn, the A fragments of slice s refilled after its group, B
    slice t after its last partner."""
    T = min(S, G)
    last_s = {t: min(T - 1, G - 1 - t) for t in range(T)}
    seq = []
    for s in range(T):
        for t in range(T - 1, -1, -1):
            if s + t >= G:
                continue
            for mb in range(2):
                seq.append(("m", s, t, mb))
            if last_s[t] == s:
                seq.append(("r", "b", t, 0))
        for mb in range(2):
            seq.append(("r", "a", s, mb))
    reads = [x for x in seq if x[0] == "r"]
    ns = min(NSPARE, len(reads) - 1)
    spare = reads[len(reads) - ns:]
    seq = [x for x in seq if x not in spare]
    lines = ["s_nop 4"]
    pending = list(enumerate(spare))

    def rd(kind, j, mb, dst):
        if kind == "a":
            return "ds_read_b128 %%[%s], %%[pa] offset:%%[oa%dm%d]" % (dst, j, mb)
        return "ds_read_b128 %%[%s], %%[pb] offset:%%[ob%d]" % (dst, j)

    for x in seq:
        if x[0] == "m":
            _, s_, t, mb = x
            lines.append("v_mfma_i32_32x32x32_i8 %%[c%dm%d], %%[a%dm%d], %%[b%d], %%[c%dm%d]" % (s_ + t, mb, s_, mb, t, s_ + t, mb))
            if pending:
                k, (_, kind, j, mb2) = pending.pop(0)
                lines.append(rd(kind, j, mb2, "x%d" % k))
        else:
            _, kind, j, mb = x
            lines.append(rd(kind, j, mb, ("a%dm%d" % (j, mb)) if kind == "a" else ("b%d" % j)))
    for k, (_, kind, j, mb) in pending:
        lines.append(rd(kind, j, mb, "x%d" % k))
    lines.append("s_waitcnt lgkmcnt(0)")
    return lines, T, [(kind, j, mb) for (_, kind, j, mb) in spare], rd


def spec2(S, G):
    lines, T, spare, rd = step_lines2(S, G)
    text = "".join('            "%s\\n\\t"\n' % l for l in lines).rstrip("\n")
    frag = (["[a%dm%d] \"+v\"(f.a[%d][%d])" % (s, mb, s, mb) for s in range(T) for mb in range(2)] +
            ["[b%d] \"+v\"(f.b[%d][0])" % (t, t) for t in range(T)])
    outs = ["[c%dm%d] \"+a\"(acc[%d][%d][0])" % (g, mb, g, mb) for g in range(G) for mb in range(2)] + frag
    outs += ["[x%d] \"=&v\"(x[%d])" % (k, k) for k in range(len(spare))]
    moves = "".join("        f.%s[%d][%d] = x[%d];\n" % (kind, j, mb if kind == "a" else 0, k)
                    for k, (kind, j, mb) in enumerate(spare))
    addr = ['[pa] "v"(pa)', '[pb] "v"(pb)']
    addr += ["[oa%dm%d] \"i\"(%d * OA + %d)" % (s, mb, s, mb * 512) for s in range(T) for mb in range(2)]
    addr += ["[ob%d] \"i\"(%d * OB)" % (t, t) for t in range(T)]
    rlines = ([rd("a", s, mb, "a%dm%d" % (s, mb)) for s in range(T) for mb in range(2)] +
              [rd("b", t, 0, "b%d" % t) for t in range(T)] + ["s_waitcnt lgkmcnt(0)"])
    rtext = "".join('            "%s\\n\\t"\n' % l for l in rlines).rstrip("\n")
    rfrag = [x.replace('"+v"', '"=v"') for x in frag]
    j = ",\n              ".join
    return """template <>
struct AsmStep2<%d, %d> {
    static constexpr bool available = true;
    template <int OA, int OB, typename F>
    __device__ __forceinline__ static void run(v16i (&acc)[%d][2][1], F &f, unsigned pa, unsigned pb) {
        v4i x[%d];
        asm volatile(
%s
            : %s
            : %s
            : "memory");
%s    }
    template <int OA, int OB, typename F>
    __device__ __forceinline__ static void read(F &f, unsigned pa, unsigned pb) {
        asm volatile(
%s
            : %s
            : %s
            : "memory");
    }
};
""" % (S, G, G, max(len(spare), 1), text, j(outs), j(addr), moves, rtext, j(rfrag), j(addr))


def main():
    out = ["// Generated by gen_asm_steps.py; do not edit.",
           "// One K block of the pair GEMM per (S, G) for waves owning one 32 x 32",
           "// output block: the kept slice-pair MFMAs of the current block, each",
           "// fragment register refilled from LDS with the next block's fragment once",
           "// its last MFMA of this block has issued (the last few refills go to spare",
           "// registers read early and moved into place after the block), and a final",
           "// wait for those reads.",
           "// OA / OB: byte distance between the LDS runs of consecutive A / B slices.",
           "#pragma once",
           "",
           "namespace oz {",
           "namespace pair {",
           "",
           "template <int S, int G>",
           "struct AsmStep {",
           "    static constexpr bool available = false;",
           "};",
           ""]
    for S in range(2, 9):
        for G in sorted({S, S + 1, 2 * S - 1}):
            out.append(spec(S, G))
    out += ["// The same for waves owning two 32 x 32 blocks stacked in M (the 128 x 64",
            "// tile of four waves at one wave per SIMD), accumulators in the",
            "// accumulation registers: built for G = 7 and 8, where the register file",
            "// of two waves per SIMD does not hold them.",
            "template <int S, int G>",
            "struct AsmStep2 {",
            "    static constexpr bool available = false;",
            "};",
            ""]
    for S in range(2, 9):
        for G in sorted({S, S + 1, 2 * S - 1}):
            if G in (7, 8):
                out.append(spec2(S, G))
    out += ["}  // namespace pair", "}  // namespace oz", ""]
    with open(os.path.join(HERE, "asm_steps.h"), "w") as fh:
        fh.write("\n".join(out))


if __name__ == "__main__":
    main()
