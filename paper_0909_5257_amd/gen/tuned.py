"""Per-process planner settings chosen by measurement (python -m paper_0909_5257_amd.tune).

Timed on one MI355X: 262144 events per launch, seeded RAMBO events with sqrt(s) U[300, 2000]
GeV and the jet cuts; ms = mean of three launches with the setting, default_ms = without it."""

TUNED = {
    ('g g > g g g g', 'double'): {'budget': 256, 'ms': 12.019, 'default_ms': 20.41},
    ('g g > g g g g', 'float'): {'externals': 'group', 'budget': 208, 'ms': 6.869, 'default_ms': 7.825},
    # measured with the first-seen class plan and 65536 events per launch (its candidates compile for a
    # quarter of an hour each); kept since
    ('g g > g g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 270.9, 'default_ms': 402.1},
    ('u g > u g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 2.767, 'default_ms': 3.495},
    ('u u > u u g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 0.846, 'default_ms': 0.978},
    ('u u > u u g g', 'float'): {'externals': 'group', 'budget': 176, 'waves_per_cu': 4, 'ms': 0.621, 'default_ms': 0.753},
    ('u u > u u g g g', 'double'): {'budget': 224, 'ms': 24.759, 'default_ms': 26.926},
    ('u u > u u g g g', 'float'): {'budget': 144, 'ms': 15.804, 'default_ms': 17.059},
    ('u u~ > g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 2.791, 'default_ms': 3.516},
    # budget scan on the final code (ms per 262144 events): 224 82.5, 240 75.8, 256 75.5, 264 71.3,
    # 272 68.8, 280 81.7, 288 98.5
    ('u u~ > g g g g g', 'double'): {'budget': 272, 'ms': 68.774, 'default_ms': 105.954},
    ('u u~ > g g g g g', 'float'): {'externals': 'group', 'budget': 208, 'ms': 43.299, 'default_ms': 47.8},
}
