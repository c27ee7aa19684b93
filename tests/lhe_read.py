"""Reader for the LHE files the tests write (XML via the standard library;
the event records are whitespace-separated numbers)."""
import xml.etree.ElementTree as ET

import numpy as np


def read(path):
    root = ET.parse(path).getroot()
    init = root.find("init").text.split()
    events = []
    for ev in root.findall("event"):
        lines = [l.split() for l in ev.text.strip().splitlines()]
        head = lines[0]
        parts = lines[1:]
        assert int(head[0]) == len(parts)
        events.append(dict(nup=int(head[0]), proc=int(head[1]), weight=float(head[2]), scale=float(head[3]),
                           aqed=float(head[4]), aqcd=float(head[5]),
                           pdg=[int(p[0]) for p in parts], status=[int(p[1]) for p in parts],
                           mothers=[(int(p[2]), int(p[3])) for p in parts],
                           colour=[(int(p[4]), int(p[5])) for p in parts],
                           p=np.array([[float(p[9]), float(p[6]), float(p[7]), float(p[8])] for p in parts]),
                           mass=np.array([float(p[10]) for p in parts]),
                           spin=[int(p[12]) for p in parts]))
    return root, init, events
