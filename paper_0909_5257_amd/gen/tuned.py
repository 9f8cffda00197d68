"""Per-process planner settings chosen by measurement (python -m paper_0909_5257_amd.tune).

Timed on one MI355X: 262144 events per launch, seeded RAMBO events with sqrt(s) U[300, 2000]
GeV and the jet cuts; ms = mean of three launches with the setting, default_ms = without it."""

TUNED = {
    ('g g > g g g g', 'double'): {'budget': 224, 'ms': 18.116, 'default_ms': 23.504},
    ('g g > g g g g', 'float'): {'budget': 160, 'ms': 11.544, 'default_ms': 12.242},
    # measured with the first-seen class plan and 65536 events per launch (its candidates compile for a
    # quarter of an hour each); kept since
    ('g g > g g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 270.9, 'default_ms': 402.1},
    ('u g > u g g g', 'double'): {'budget': 224, 'ms': 4.086, 'default_ms': 4.57},
    ('u u > u u g g', 'double'): {'budget': 160, 'ms': 1.344, 'default_ms': 1.414},
    ('u u > u u g g', 'float'): {'externals': 'group', 'budget': 176, 'waves_per_cu': 4, 'ms': 0.785, 'default_ms': 0.965},
    ('u u > u u g g g', 'double'): {'budget': 224, 'ms': 26.554, 'default_ms': 28.575},
    ('u u > u u g g g', 'float'): {'externals': 'group', 'budget': 176, 'ms': 17.466, 'default_ms': 19.388},
    ('u u~ > g g g g', 'double'): {'budget': 224, 'ms': 4.093, 'default_ms': 4.606},
    ('u u~ > g g g g g', 'double'): {'budget': 224, 'ms': 120.778, 'default_ms': 145.847},
    ('u u~ > g g g g g', 'float'): {'externals': 'group', 'budget': 208, 'ms': 67.996, 'default_ms': 72.29},
}
