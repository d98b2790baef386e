"""Recipe that wrote the text fixtures in this folder from the paper's LaTeX.

The paper prints the data behind two of its figures as pgfplots coordinate
lists.  This script pulls those lists out of the paper's source and writes
them as plain whitespace-separated text, one value per line, so the oracle's
tests can check themselves against numbers the paper prints.  It is run once
by hand; no test runs it, and nothing here computes anything of the method.

    python tests/golden/extract_figure_data.py <the paper's LaTeX source>

(the source holds the coordinate lists of Fig. "Transmittance comparison"
and Fig. "Blending comparison" (a) as pgfplots data).

Fixtures written:
  fig_transmittance_dots.txt    Fig. "Transmittance comparison", blue dots:
                                discrete transmittance after every 5 splats.
  fig_transmittance_mother.txt  same figure, green curves: the mother T(tau).
  fig_blending_concentric.txt   Fig. "Blending comparison" (a), the centre
                                scan-line of 3 concentric Gaussians: per-splat
                                contributions (red, green, blue) and their sum.
"""
import re
import sys
from pathlib import Path

# Panel file stem -> operator name used by the oracle's operator table.
PANELS = {
    "PowermLaw_v2": "powerlaw_v2",
    "Exponential": "exponential",
    "Quadratic_cm0p5": "quadratic_c-0.5",
    "citetvicini2021non_gamma0p5": "vicini_g0.5",
    "Blend_gamma0p5": "blended_g0.5",
    "Linear": "linear",
    "Quadratic_c0p5": "quadratic_c0.5",
    "Quadratic_c1": "quadratic_c1",
    "PowermLaw_vm1": "powerlaw_vm1",
}

FILE_RE = re.compile(r"^%% file: (\S+)")
PLOT_RE = re.compile(r"\\addplot\[([^\]]*)\] coordinates \{(.*)\};")
PAIR_RE = re.compile(r"\(([-0-9.eE]+),([-0-9.eE]+)\)")


def main(paper):
    lines = Path(paper).read_text().splitlines()
    current = None
    trans_dots, trans_mother, blend = [], [], []
    for lineno, line in enumerate(lines, 1):
        m = FILE_RE.match(line)
        if m:
            current = m.group(1)
            continue
        p = PLOT_RE.search(line)
        if not p or current is None:
            continue
        style, body = p.group(1), p.group(2)
        pairs = PAIR_RE.findall(body)
        stem = Path(current).stem
        if stem.startswith("n100_random_center_prob_"):
            op = PANELS[stem[len("n100_random_center_prob_"):]]
            if style.startswith("blue"):
                trans_dots += [(op, x, y, lineno) for x, y in pairs]
            elif style.startswith("green"):
                trans_mother += [(op, x, y, lineno) for x, y in pairs]
        elif stem.startswith("n3_concentric_cross_section_"):
            op = PANELS[stem[len("n3_concentric_cross_section_"):]]
            curve = {"red": "red", "green!70!black": "green", "blue": "blue",
                     "black": "sum"}[style.split(",")[0]]
            blend += [(op, curve, x, y, lineno) for x, y in pairs]
    out = Path(__file__).parent
    src = ("# Source: Sec. 4 (Evaluation), Fig. 'Transmittance comparison' "
           "(100 splats, opacity 0.02).\n")
    (out / "fig_transmittance_dots.txt").write_text(
        src + "# Blue dots: discrete transmittance after every 5 splats.\n"
        "# operator tau_bar T_bar\n"
        + "".join(f"{o} {x} {y}\n" for o, x, y, _ in trans_dots))
    (out / "fig_transmittance_mother.txt").write_text(
        src + "# Green curves: the mother transmittance T(tau).\n"
        "# operator tau T\n"
        + "".join(f"{o} {x} {y}\n" for o, x, y, _ in trans_mother))
    rows = {}
    for o, c, x, y, _ in blend:
        rows.setdefault((o, x), {})[c] = y
    (out / "fig_blending_concentric.txt").write_text(
        "# Source: Sec. 4 (Evaluation), Fig. 'Blending comparison' (a): "
        "3 concentric Gaussians,\n# opacity 1, red in front, then green, "
        "blue at the back; centre scan-line.\n"
        "# Columns: per-splat contribution E_i*p_i of each splat and their "
        "sum, at pixel x.\n# operator x red green blue sum\n"
        + "".join(f"{o} {x} {v['red']} {v['green']} {v['blue']} {v['sum']}\n"
                  for (o, x), v in rows.items()))
    print(len(trans_dots), len(trans_mother), len(blend))


if __name__ == "__main__":
    main(sys.argv[1])
