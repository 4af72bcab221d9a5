"""Writes fig1_drag_error.json: the six curves of Fig. 1 of the paper (relative
error C/C_ref - 1 of the dimensionless drag on a simple-cubic periodic sphere
array, L = 32, D = 16, a = 1e-5, Sec. 3), read back from the vector coordinates
of the figure's pgf source.

Each curve is matched to its legend label by stroke colour; the data axis is
calibrated from the y tick labels (-0.2 ... 0.2) and the tau tick labels on the
top axis.  Run:  python tests/golden/extract_fig1.py <text of the paper holding
the figure's pgf source>
"""
import json
import os
import re
import sys

NUM = r"(-?[0-9.]+)in"


def main(path):
    lines = open(path, encoding="utf-8").read().splitlines()
    start = next(i for i, l in enumerate(lines) if "plot_tau_DragForce_error" in l or "DragForceError" in l)
    body = lines[start - 10: start + 1400] if start > 10 else lines
    text = "\n".join(body)
    # y calibration from right-aligned tick labels
    yt = re.findall(r"pgftext\[x=[0-9.]+in,y=([0-9.]+)in,right,\]\{[^}]*\}\{[^}]*\}\\selectfont ([^}]+)\}", text)
    ys = [(float(y), float(lbl.replace("\u2212", "-"))) for y, lbl in yt]
    (y0, v0), (y1, v1) = ys[0], ys[-1]
    yscale = (v1 - v0) / (y1 - y0)
    # tau calibration from the top-axis labels (placed at y above the axes, 'bottom')
    tt = re.findall(r"pgftext\[x=([0-9.]+)in,y=[0-9.]+in,,bottom\]\{[^}]*\}\{[^}]*\}\\selectfont ([0-9.]+)\}", text)
    (x0, t0), (x1, t1) = (float(tt[0][0]), float(tt[0][1])), (float(tt[-1][0]), float(tt[-1][1]))
    # legend: label -> fill colour of the marker drawn just before it
    legend = {}
    for m in re.finditer(r"selectfont ((?:MEM|PSM) [A-Z0-9]+)\}", text):
        before = text[:m.start()]
        col = re.findall(r"definecolor\{currentfill\}\{rgb\}\{([0-9.,]+)\}", before)[-1]
        legend[col] = m.group(1)
    # data series: stroked paths with >= 8 points inside the axes
    out = {}
    for blk in re.split(r"\\begin\{pgfscope\}", text):
        cm = re.search(r"definecolor\{currentstroke\}\{rgb\}\{([0-9.,]+)\}", blk)
        pts = re.findall(r"pgfpath(?:moveto|lineto)\{\\pgfqpoint\{" + NUM + r"\}\{" + NUM + r"\}\}", blk)
        if not cm or cm.group(1) not in legend or len(pts) != 8:
            continue
        label = legend[cm.group(1)]
        if label in out:
            continue
        series = []
        for xs, ysv in pts:
            tau = t0 + (float(xs) - x0) * (t1 - t0) / (x1 - x0)
            err = v0 + (float(ysv) - y0) * yscale
            series.append([round(tau, 4), round(err, 5)])
        out[label] = series
    doc = {
        "source": "Fig. 1 of arXiv:1702.04910 (Sec. 3, force on a fixed sphere in Stokes flow): C/C_ref - 1, "
                  "C_ref = 2.8402; SC array L = 32, D = L/2, a = 1e-5; MEM with TRT, Lambda = 3/16; PSM BGK-based. "
                  "Values read back from the figure's vector coordinates (read-back precision about 1e-5).",
        "series": out,
    }
    dst = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig1_drag_error.json")
    with open(dst, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: extract_fig1.py <paper text holding the pgf source of Fig. 1>")
    main(sys.argv[1])
