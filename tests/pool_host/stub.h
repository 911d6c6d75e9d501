#pragma once
void stub_count_create();
int stub_creates();
int stub_report();
