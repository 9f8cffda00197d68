"""Per-process planner settings chosen by measurement (python -m paper_0909_5257_amd.tune).

Timed on one MI355X: 262144 events per launch, seeded RAMBO events with sqrt(s) U[300, 2000]
GeV and the jet cuts; ms = mean of three launches with the setting, default_ms = without it."""

TUNED = {
    ('g g > g g g g', 'double'): {'budget': 192, 'ms': 23.162, 'default_ms': 28.289},
    # measured with the first-seen class plan and 65536 events per launch (its candidates compile for a
    # quarter of an hour each); kept under the greedy plan
    ('g g > g g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 270.9, 'default_ms': 402.1},
    ('u g > u g g g', 'double'): {'budget': 192, 'ms': 4.534, 'default_ms': 5.403},
    ('u u > u u g g', 'float'): {'externals': 'group', 'budget': 176, 'waves_per_cu': 4, 'ms': 0.833, 'default_ms': 1.003},
    ('u u > u u g g g', 'float'): {'budget': 160, 'ms': 17.878, 'default_ms': 19.443},
    ('u u~ > g g g g', 'double'): {'budget': 192, 'ms': 4.589, 'default_ms': 5.413},
    ('u u~ > g g g g g', 'double'): {'budget': 224, 'ms': 137.007, 'default_ms': 156.558},
}
